"""GPU parity of ends-free alignment (free pattern / text prefixes and
suffixes, semi-global read-in-reference alignment) against the CPU oracle:
scores and CIGAR runs byte for byte, through the C ABI."""
import numpy as np
import pytest

from gpu_util import assert_same, say

pytestmark = pytest.mark.gpu

PEN = (4, 6, 2)


@pytest.fixture(scope="module")
def wfa():
    import paper_2204_02085_amd as w

    return w


@pytest.fixture(scope="module")
def aligner(wfa):
    al = wfa.Aligner(0)
    yield al
    al.close()


@pytest.fixture(autouse=True)
def _defaults(aligner):
    aligner.set_options()
    aligner.set_ends_free()
    yield
    aligner.set_options()
    aligner.set_ends_free()


def oracle_of(oracle_lib, batch, ends, pen=PEN, cigar=True):
    return oracle_lib.align_batch(batch, pen, cigar=cigar, threads=8, ends=ends)


def flanked(synth_lib, batch, seed, lo, hi):
    """The batch with random flanks of lo..hi bases added to both ends of
    every text (a read inside a stretch of reference)."""
    rng = np.random.default_rng(seed)
    pairs = []
    for i in range(len(batch)):
        p, t = batch.pair(i)
        a = rng.choice(list(b"ACGT"), int(rng.integers(lo, hi + 1))).astype(np.uint8).tobytes()
        b = rng.choice(list(b"ACGT"), int(rng.integers(lo, hi + 1))).astype(np.uint8).tobytes()
        pairs.append((p, a + t + b))
    return synth_lib.from_pairs(pairs)


ENDS = [(5, 0, 0, 5), (0, 10, 10, 0), (20, 20, 20, 20), (3, 7, 2, 9), (100, 100, 0, 0)]


@pytest.mark.parametrize("ends", ENDS)
def test_pairs100_e4(aligner, oracle_lib, synth_lib, ends):
    say(f"case: ends-free {ends}, pairs100_e4 3000 pairs, CIGAR")
    b = synth_lib.workload("pairs100_e4_5m", 3000, first=901)
    aligner.set_ends_free(*ends)
    got = aligner.align(b, PEN)
    assert_same(got, oracle_of(oracle_lib, b, ends), b, f"ends {ends}")


@pytest.mark.parametrize("ends", [(0, 0, 10_000, 10_000), (0, 0, 30, 30)])
def test_semi_global_read_in_reference(aligner, oracle_lib, synth_lib, ends):
    """100 bp reads with 4 % edits inside 110-200 bp of reference."""
    say(f"case: semi-global {ends}, reads in flanked references")
    b = flanked(synth_lib, synth_lib.workload("pairs100_e4_5m", 2000, first=55), 7, 5, 50)
    aligner.set_ends_free(*ends)
    got = aligner.align(b, PEN)
    ref = oracle_of(oracle_lib, b, ends)
    assert_same(got, ref, b, f"semi-global {ends}")
    if ends[2] >= 50:  # fully free text ends: the read's own edits only
        assert int(np.median(ref.scores)) <= 40


def test_uneven_score_only_and_penalties(aligner, oracle_lib, synth_lib):
    say("case: ends-free (8, 4, 6, 12), uneven 50-300 bp, score only and (1, 0, 1)")
    b = synth_lib.workload("uneven50_300_2m", 2000, first=3)
    ends = (8, 4, 6, 12)
    aligner.set_ends_free(*ends)
    sc, _, _ = aligner.align(b, PEN, cigar=False)
    assert np.array_equal(sc, oracle_of(oracle_lib, b, ends, cigar=False).scores)
    got = aligner.align(b, (1, 0, 1))
    assert_same(got, oracle_of(oracle_lib, b, ends, pen=(1, 0, 1)), b, "edit distance ends-free")


def test_host_memory_chunks(aligner, oracle_lib, synth_lib):
    say("case: ends-free (0, 0, 40, 40) through the host-memory pipeline, chunks of 500")
    b = flanked(synth_lib, synth_lib.workload("pairs100_e2_5m", 2500, first=11), 3, 0, 40)
    ends = (0, 0, 40, 40)
    aligner.set_ends_free(*ends)
    aligner.set_options(host_chunk_pairs=500)
    got = aligner.align_host(b, PEN)
    assert_same(got, oracle_of(oracle_lib, b, ends), b, "ends-free host")


def test_edge_cases(aligner, oracle_lib, synth_lib):
    say("case: ends-free edge cases (empty sides, all free, equal sequences)")
    pairs = [(b"", b""), (b"", b"ACGT"), (b"ACGT", b""), (b"ACGT", b"ACGT"), (b"A", b"C"),
             (b"ACGTACGT", b"TTTTACGTACGTTTTT"), (b"GGGGACGT", b"ACGTCCCC"),
             (b"ACGT" * 10, b"TGCA" * 10)]
    b = synth_lib.from_pairs(pairs)
    for ends in [(0, 0, 4, 4), (2, 2, 2, 2), (50, 50, 50, 50), (0, 4, 4, 0)]:
        aligner.set_ends_free(*ends)
        got = aligner.align(b, PEN)
        assert_same(got, oracle_of(oracle_lib, b, ends), b, f"edges {ends}")


def test_back_to_global(aligner, oracle_lib, synth_lib):
    """Clearing the free ends restores global alignment on the same context."""
    say("case: ends-free then global on one context")
    b = synth_lib.workload("pairs100_e4_5m", 2000, first=5)
    aligner.set_ends_free(10, 10, 10, 10)
    aligner.align(b, PEN)
    aligner.set_ends_free()
    got = aligner.align(b, PEN)
    assert_same(got, oracle_lib.align_batch(b, PEN, cigar=True, threads=8), b, "global again")


SHAPES = [(32, 8), (48, 16), (64, 16), (64, 32), (128, 64), (256, 64)]


@pytest.mark.parametrize("window,lanes", SHAPES)
def test_short_kernel_shapes(aligner, oracle_lib, synth_lib, wfa, window, lanes):
    """Free ends inside the short kernel's window, for each of several
    shapes, int8 (100 bp) and int16 (50-300 bp) offsets, score and CIGAR:
    the short kernel finishes most pairs (windows up to 128) and every
    result is the oracle's."""
    ends = (6, 3, 4, 9)
    aligner.set_ends_free(*ends)
    for name, count in (("pairs100_e4_5m", 3000), ("uneven50_300_2m", 1500)):
        say(f"case: ends-free {ends}, short kernel W{window} G{lanes}, {name}")
        b = synth_lib.workload(name, count, first=77)
        aligner.set_options(window=window, lanes_per_pair=lanes,
                            schedule=wfa.WFA_SCHED_PERSISTENT)
        got = aligner.align(b, PEN)
        st = aligner.stats()
        assert_same(got, oracle_of(oracle_lib, b, ends), b, f"W{window} G{lanes} {name}")
        if name == "pairs100_e4_5m" and window <= 128:  # (a 256-wide CIGAR plan needs more LDS)
            assert st["short_pairs"] > count // 2, st
        sc, _, _ = aligner.align(b, PEN, cigar=False)
        assert np.array_equal(sc, oracle_of(oracle_lib, b, ends, cigar=False).scores)


def test_short_kernel_semi_global(aligner, oracle_lib, synth_lib, wfa):
    """Reads inside references a few bases longer, text ends free: the short
    kernel holds the free start diagonals; plain and persistent launches."""
    b = flanked(synth_lib, synth_lib.workload("pairs100_e4_5m", 3000, first=2024), 9, 0, 8)
    ends = (0, 0, 16, 16)
    aligner.set_ends_free(*ends)
    ref = oracle_of(oracle_lib, b, ends)
    for sched in ("PLAIN", "PERSISTENT", "AUTO"):
        say(f"case: semi-global short kernel, schedule {sched}")
        aligner.set_options(schedule=getattr(wfa, "WFA_SCHED_" + sched))
        got = aligner.align(b, PEN)
        assert aligner.stats()["short_pairs"] > 1500
        assert_same(got, ref, b, f"semi-global {sched}")


def test_full_size_ends_free(aligner, oracle_lib, synth_lib):
    """5,000,000 pairs of 100 bp at E = 4 % aligned with 10 free bases at
    each end of either sequence, default launch: every pair's runs spell
    both sequences; a sample (random pairs, the 500 highest scores, the
    first and last pair) is byte-exact against the oracle and its CIGARs
    re-score to the ends-free score."""
    import brute

    ends = (10, 10, 10, 10)
    b = synth_lib.workload("pairs100_e4_5m")
    say(f"case: pairs100_e4_5m full size, ends-free {ends}")
    aligner.set_ends_free(*ends)
    sc, runs, off = aligner.align(b, PEN, capacity=len(b) * 40 + 1024)
    st = aligner.stats()
    say(f"  stats: {st}")
    assert st["short_pairs"] > 0.99 * len(b)
    # spelling: the runs consume exactly n pattern and m text bases
    counts = np.diff(off.astype(np.int64))
    ops = (runs & 15).astype(np.int64)
    lens = (runs >> 4).astype(np.int64)
    pid = np.repeat(np.arange(len(b)), counts)
    assert not ((pid[1:] == pid[:-1]) & (ops[1:] == ops[:-1])).any()
    used_p = np.bincount(pid, weights=lens * (ops != 2), minlength=len(b)).astype(np.int64)
    used_t = np.bincount(pid, weights=lens * (ops != 3), minlength=len(b)).astype(np.int64)
    assert np.array_equal(used_p, b.p_len.astype(np.int64))
    assert np.array_equal(used_t, b.t_len.astype(np.int64))
    rng = np.random.default_rng(3)
    top = np.argsort(sc, kind="stable")[-500:]
    idx = np.unique(np.concatenate([rng.choice(len(b), 20_000, replace=False), top,
                                    [0, len(b) - 1]]))
    sub = b.subset(idx)
    ref = oracle_of(oracle_lib, sub, ends)
    sub_off = np.zeros(len(idx) + 1, np.uint64)
    pieces = [runs[int(off[i]):int(off[i + 1])] for i in idx]
    np.cumsum([len(p) for p in pieces], out=sub_off[1:])
    got = (sc[idx], np.concatenate(pieces).astype(np.uint32), sub_off)
    assert_same(got, ref, sub, "full-size ends-free sample")
    for j in range(0, len(idx), 40):
        p, t = sub.pair(j)
        r = got[1][int(sub_off[j]):int(sub_off[j + 1])]
        assert brute.check_cigar_ends(p, t, r, *PEN, ends) == int(got[0][j])
