"""GPU parity of the WF-adaptive heuristic (wavefront reduction) against the
CPU oracle's reduction: scores and CIGAR runs element by element, through
the C ABI, on short, uneven and long pairs, tight and loose thresholds."""
import ctypes

import numpy as np
import pytest

import brute
from gpu_util import assert_same, runs_of, say

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
    aligner.set_heuristic()
    yield
    aligner.set_options()
    aligner.set_ends_free()
    aligner.set_heuristic()


def oracle_of(oracle_lib, batch, ad, pen=PEN, cigar=True):
    slot = int((batch.p_len.astype(np.int64) + batch.t_len.astype(np.int64)).max(initial=0)) + 1
    return oracle_lib.align_batch(batch, pen, cigar=cigar, threads=8, adaptive=ad, slot=slot)


def test_worked_example(aligner, oracle_lib, synth_lib):
    """The hand-derived cases (AA / CCAA and its mirror, AC / CAC)."""
    say("case: adaptive worked example")
    cases = [((1, 0), b"AA", b"CCAA", 14, "1X2I1M"), ((7, 0), b"AA", b"CCAA", 14, "1X2I1M"),
             ((8, 0), b"AA", b"CCAA", 10, "2I2M"), ((1, 1), b"AA", b"CCAA", 10, "2I2M"),
             ((1, 0), b"CCAA", b"AA", 14, "1X2D1M"), ((1, 0), b"AC", b"CAC", 8, "1I2M")]
    for ad, p, t, score, cigar in cases:
        aligner.set_heuristic(*ad)
        b = synth_lib.from_pairs([(p, t)])
        sc, runs, off = aligner.align(b, PEN)
        assert int(sc[0]) == score, (ad, p, t)
        assert oracle_lib.cigar_string(runs[int(off[0]):int(off[1])]) == cigar, (ad, p, t)


@pytest.mark.parametrize("ad", [(1, 0), (3, 1), (5, 5), (10, 50), (20, 2)])
@pytest.mark.parametrize("pen", [(4, 6, 2), (1, 0, 1), (2, 3, 1)])
def test_random_pairs(aligner, oracle_lib, synth_lib, ad, pen):
    """Related and unrelated pairs of 0-300 bases, CIGAR and score only."""
    say(f"case: adaptive {ad} penalties {pen}, random pairs")
    rng = np.random.default_rng(sum(ad) * 31 + sum(pen))
    pairs = synth_lib.random_pairs(rng, 300, 120) + synth_lib.random_pairs(rng, 60, 300)
    pairs += synth_lib.random_pairs(rng, 40, 80, related=False)
    pairs += [(b"", b""), (b"", b"ACGT"), (b"TTG", b""), (b"A", b"A"), (b"AC", b"CA")]
    b = synth_lib.from_pairs(pairs)
    aligner.set_heuristic(*ad)
    got = aligner.align(b, pen)
    ref = oracle_of(oracle_lib, b, ad, pen)
    assert_same(got, ref, b, f"adaptive {ad} {pen}")
    # each CIGAR spells its pair and costs between the optimum and the score
    # (a gap reopened right after closing merges into one run)
    exact = oracle_lib.align_batch(b, pen, cigar=False, threads=8).scores
    for i in range(len(b)):
        c = brute.check_cigar(*b.pair(i), runs_of(got[1], got[2], i), *pen)
        assert int(exact[i]) <= c <= int(got[0][i]), i
    sc = aligner.align(b, pen, cigar=False)[0]
    assert np.array_equal(sc, ref.scores)


@pytest.mark.parametrize("ad", [(1, 0), (4, 2), (10, 50)])
def test_pairs100_and_uneven(aligner, oracle_lib, synth_lib, ad):
    """The 100 bp read pairs at E = 4 % and uneven 50-300 bp pairs."""
    say(f"case: adaptive {ad}, pairs100_e4 + uneven50_300")
    e4 = synth_lib.workload("pairs100_e4_5m", 4000, first=77)
    un = synth_lib.workload("uneven50_300_2m", 2000, first=5)
    b = synth_lib.from_pairs([e4.pair(i) for i in range(len(e4))] +
                             [un.pair(i) for i in range(len(un))])
    aligner.set_heuristic(*ad)
    got = aligner.align(b, PEN)
    ref = oracle_of(oracle_lib, b, ad)
    assert_same(got, ref, b, f"adaptive {ad}")
    st = aligner.stats()
    assert st["general_pairs"] == len(b) and st["short_pairs"] == 0
    exact = oracle_lib.align_batch(b, PEN, cigar=False, threads=8).scores
    assert (ref.scores >= exact).all()


@pytest.mark.parametrize("ad", [(10, 50), (5, 3), (1, 0)])
@pytest.mark.parametrize("cigar", [True, False])
def test_long_reads(aligner, oracle_lib, synth_lib, ad, cigar):
    """1-10 kbp pairs at 5-10 % events (the 16-bit and, past 32767 bases,
    32-bit ring rows are covered by the kernel's other tests)."""
    say(f"case: adaptive {ad}, long reads, cigar={cigar}")
    b = synth_lib.workload("long1k_10k_100k", 48, first=300)
    aligner.set_heuristic(*ad)
    cap = int((b.p_len.astype(np.int64) + b.t_len).sum()) + 16
    got = aligner.align(b, PEN, cigar=cigar, capacity=cap if cigar else None)
    ref = oracle_of(oracle_lib, b, ad, cigar=cigar)
    assert_same(got, ref, b, f"adaptive long {ad}")


def test_no_reduction_is_exact(aligner, oracle_lib, synth_lib):
    """A minimum width above any wavefront's span: the exact alignment."""
    say("case: adaptive without reduction equals exact")
    b = synth_lib.workload("uneven50_300_2m", 3000, first=999)
    aligner.set_heuristic(1 << 20, 0)
    got = aligner.align(b, PEN)
    assert_same(got, oracle_lib.align_batch(b, PEN, threads=8), b, "no reduction")


def test_settings_and_errors(aligner, wfa, oracle_lib, synth_lib):
    say("case: adaptive settings and errors")
    with pytest.raises(wfa.WFAError):
        aligner.set_heuristic(-1, 0)
    with pytest.raises(wfa.WFAError):
        aligner.set_heuristic(5, -2)
    aligner.set_heuristic(3, 1)
    with pytest.raises(wfa.WFAError):
        aligner.set_ends_free(0, 0, 5, 5)
    aligner.set_heuristic()
    aligner.set_ends_free(0, 0, 5, 5)
    with pytest.raises(wfa.WFAError):
        aligner.set_heuristic(3, 1)
    aligner.set_ends_free()
    # back to exact: the short kernels take the batch again
    b = synth_lib.workload("pairs100_e4_5m", 2000, first=3)
    aligner.set_heuristic(1, 0)
    aligner.set_heuristic()
    got = aligner.align(b, PEN)
    assert_same(got, oracle_lib.align_batch(b, PEN, threads=8), b, "exact again")
    assert aligner.stats()["short_pairs"] > 0


def test_noalloc_entry_point(aligner, wfa, oracle_lib, synth_lib):
    """The allocation-free entry point follows the context's heuristic."""
    import torch

    say("case: adaptive through the allocation-free entry point")
    b = synth_lib.workload("uneven50_300_2m", 2000, first=42)
    aligner.set_heuristic(2, 1)
    pat, txt, pairs = aligner.to_device(b)
    cap = len(b) * 80 + 1024
    scores, runs, offsets = aligner.alloc_outputs(len(b), cap)
    needed = ctypes.c_size_t(0)
    bad = ctypes.c_int64(-1)
    rc = wfa.wfa_align_batch_noalloc(aligner.ctx, pat.data_ptr(), txt.data_ptr(),
                                     pairs.data_ptr(), len(b), wfa.WFA_ASCII,
                                     wfa.wfa_penalties(*PEN), wfa.WFA_CIGAR, scores.data_ptr(),
                                     runs.data_ptr(), cap, offsets.data_ptr(),
                                     ctypes.byref(needed), ctypes.byref(bad), None)
    torch.cuda.synchronize()
    assert rc == wfa.WFA_OK, (rc, bad.value)
    got = (scores.cpu().numpy(), runs[: needed.value].cpu().numpy().view(np.uint32),
           offsets.cpu().numpy().view(np.uint64))
    assert_same(got, oracle_of(oracle_lib, b, (2, 1)), b, "noalloc adaptive")
