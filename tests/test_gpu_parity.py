"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Scores and CIGAR runs must be byte-identical to the oracle's.  Inputs are
the seeded synthetic workloads (pairs of 100 bp reads at 2 % and 4 % edits,
uneven 50-300 bp pairs, long 1-10 kbp pairs) plus edge cases.
"""
import os

import numpy as np
import pytest

import brute
from gpu_util import assert_same, check_invariants_vectorized, check_sample_cigars, say

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
    yield
    aligner.set_options()


def oracle_of(oracle_lib, batch, pen=PEN, cigar=True):
    return oracle_lib.align_batch(batch, pen, cigar=cigar, threads=8)


def oracle_all(oracle_lib, batch, slot, pen=PEN):
    """The oracle on every pair of a full-size batch, on all host threads
    (at most 16); `slot` bounds the runs of one pair."""
    threads = max(1, min(16, os.cpu_count() or 1))
    return oracle_lib.align_batch(batch, pen, cigar=True, threads=threads, slot=slot)


@pytest.mark.parametrize("schedule", ["PLAIN", "AUTO"])
def test_pairs100_e2_10k_all(aligner, oracle_lib, synth_lib, wfa, schedule):
    """10,000 pairs of 100 bp at E = 2 %: every pair bit-exact, with the plain
    per-batch kernel and with the default (persistent) schedule."""
    say(f"case: pairs100_e2_10k, all pairs, CIGAR, schedule {schedule}")
    b = synth_lib.workload("pairs100_e2_10k")
    aligner.set_options(schedule=getattr(wfa, "WFA_SCHED_" + schedule))
    got = aligner.align(b, PEN)
    st = aligner.stats()
    assert st["short_pairs"] == len(b)
    assert st["schedule"] == getattr(wfa, "WFA_SCHED_" + ("PLAIN" if schedule == "PLAIN"
                                                          else "PERSISTENT"))
    assert_same(got, oracle_of(oracle_lib, b), b, "pairs100_e2_10k")
    check_sample_cigars(b, *got, PEN, range(0, len(b), 50))


@pytest.mark.parametrize("schedule", ["PLAIN", "PERSISTENT", "GENERAL", "AUTO"])
def test_pairs100_e4_schedules(aligner, oracle_lib, synth_lib, wfa, schedule):
    say(f"case: pairs100_e4 20k pairs, schedule {schedule}")
    b = synth_lib.workload("pairs100_e4_5m", 20_000)
    aligner.set_options(schedule=getattr(wfa, "WFA_SCHED_" + schedule))
    got = aligner.align(b, PEN)
    assert_same(got, oracle_of(oracle_lib, b), b, f"e4/{schedule}")


SHAPES = [(16, 8), (16, 16), (24, 8), (32, 32), (32, 16), (32, 8), (48, 16), (64, 64), (64, 32),
          (64, 16), (128, 64), (128, 32), (256, 64)]


@pytest.mark.parametrize("window,lanes", SHAPES)
def test_windows_identical(aligner, oracle_lib, synth_lib, wfa, window, lanes):
    """Every short-kernel shape (window, lanes per pair) gives the oracle's
    bytes: 100 bp pairs (int8 rows) and uneven 50-300 bp pairs (int16 rows,
    target diagonals far from diagonal 0, so the first layers computed are
    outer ones), in CIGAR and score mode.  Narrow windows hand most pairs to
    the general kernel."""
    say(f"case: window {window} lanes {lanes}")
    aligner.set_options(window=window, lanes_per_pair=lanes, schedule=wfa.WFA_SCHED_PLAIN)
    for name, first in [("pairs100_e4_5m", 50_000), ("uneven50_300_2m", 1000)]:
        b = synth_lib.workload(name, 3000, first=first)
        got = aligner.align(b, PEN)
        assert_same(got, oracle_of(oracle_lib, b), b, f"{name} window {window} lanes {lanes}")
        got = aligner.align(b, PEN, cigar=False)
        assert_same(got, oracle_of(oracle_lib, b, cigar=False), b,
                    f"{name} score window {window} lanes {lanes}")
        st = aligner.stats()
        assert st["window"] == window and st["lanes_per_pair"] == lanes


def test_score_only(aligner, oracle_lib, synth_lib):
    say("case: score-only mode, pairs100_e4 and uneven")
    for name, cnt in [("pairs100_e4_5m", 20_000), ("uneven50_300_2m", 5000)]:
        b = synth_lib.workload(name, cnt)
        got = aligner.align(b, PEN, cigar=False)
        assert_same(got, oracle_of(oracle_lib, b, cigar=False), b, f"score {name}")


def test_uneven_sample(aligner, oracle_lib, synth_lib):
    say("case: uneven 50-300 bp, 20k pairs, CIGAR")
    b = synth_lib.workload("uneven50_300_2m", 20_000)
    got = aligner.align(b, PEN)
    assert_same(got, oracle_of(oracle_lib, b), b, "uneven")


def test_edge_cases(aligner, oracle_lib, synth_lib):
    say("case: edge cases (empty, identical, unrelated, ragged)")
    rng = np.random.default_rng(9)
    pairs = [(b"", b""), (b"", b"ACGT"), (b"ACGTA", b""), (b"A", b"A"), (b"A", b"C"),
             (b"ACGT" * 25, b"ACGT" * 25), (b"A" * 300, b"C" * 300), (b"A" * 33, b"A" * 31),
             (b"ACGT" * 8, b"ACGT" * 8 + b"T"), (b"G" * 64, b"G" * 65)]
    pairs += synth_lib.random_pairs(rng, 200, 200)
    pairs += synth_lib.random_pairs(rng, 50, 150, related=False)
    b = synth_lib.from_pairs(pairs)
    got = aligner.align(b, PEN)
    assert_same(got, oracle_of(oracle_lib, b), b, "edge")


@pytest.mark.parametrize("pen", [(1, 0, 1), (2, 3, 1), (5, 7, 1), (3, 1, 4), (6, 4, 2)])
def test_penalty_sets(aligner, oracle_lib, synth_lib, pen):
    say(f"case: penalties {pen}")
    b = synth_lib.workload("uneven50_300_2m", 3000, first=7)
    got = aligner.align(b, pen)
    assert_same(got, oracle_of(oracle_lib, b, pen), b, f"pen {pen}")


@pytest.mark.parametrize("pen", [(4, 6, 4), (3, 1, 4), (1, 0, 1), (2, 3, 1), (5, 2, 3)])
def test_general_kernel_penalty_sets(aligner, oracle_lib, synth_lib, wfa, pen):
    """Every pair on the general kernel under penalty sets whose scaled gap
    extension exceeds one step (steps without a wavefront between steps with
    one, so the wavefront's range can narrow from one step to the next)."""
    say(f"case: general kernel, penalties {pen}")
    b = synth_lib.workload("uneven50_300_2m", 1500, first=4321)
    aligner.set_options(schedule=wfa.WFA_SCHED_GENERAL)
    got = aligner.align(b, pen)
    assert_same(got, oracle_of(oracle_lib, b, pen), b, f"general pen {pen}")
    sc, _, _ = aligner.align(b, pen, cigar=False)
    assert np.array_equal(sc, oracle_of(oracle_lib, b, pen, cigar=False).scores)


def test_host_memory_path(aligner, oracle_lib, synth_lib):
    say("case: host-memory staging path")
    b = synth_lib.workload("pairs100_e4_5m", 5000, first=1000)
    got = aligner.align_host(b, PEN)
    assert_same(got, oracle_of(oracle_lib, b), b, "host")


def test_graph_replays_match_eager(aligner, oracle_lib, synth_lib, wfa):
    """The captured-graph path, replayed several times with other device work
    in between, gives the eager path's bytes on every replay."""
    import torch

    say("case: graph replays vs eager, pairs100_e4 30k")
    b = synth_lib.workload("pairs100_e4_5m", 30_000, first=123)
    n = len(b)
    pat, txt, pairs = aligner.to_device(b)
    scores, runs, offsets = aligner.alloc_outputs(n, n * 40)
    aligner.set_options(schedule=wfa.WFA_SCHED_PERSISTENT, use_graph=-1)
    need = aligner.align_device(pat, txt, pairs, n, scores, runs, offsets)
    eager = (scores.cpu().numpy().copy(), runs[:need].cpu().numpy().copy(),
             offsets.cpu().numpy().copy())
    aligner.set_options(schedule=wfa.WFA_SCHED_PERSISTENT, use_graph=1)
    for rep in range(4):
        scores.fill_(-7)
        runs.fill_(0)
        junk = torch.randn(1 << 20, device=scores.device).sum()  # eager work between replays
        torch.cuda.synchronize()
        need2 = aligner.align_device(pat, txt, pairs, n, scores, runs, offsets)
        assert aligner.stats()["graph_replayed"] == 1
        assert need2 == need
        assert np.array_equal(scores.cpu().numpy(), eager[0]), f"replay {rep} scores"
        assert np.array_equal(runs[:need].cpu().numpy(), eager[1]), f"replay {rep} runs"
        assert np.array_equal(offsets.cpu().numpy(), eager[2]), f"replay {rep} offsets"
        del junk
    ref = oracle_of(oracle_lib, b)
    assert_same((eager[0], eager[1].view(np.uint32), eager[2].view(np.uint64)), ref, b, "eager")


def test_repeat_runs_identical(aligner, synth_lib, wfa):
    say("case: 5 repeated runs, uneven workload, byte-identical")
    b = synth_lib.workload("uneven50_300_2m", 20_000, first=999)
    first = aligner.align(b, PEN)
    for _ in range(4):
        again = aligner.align(b, PEN)
        for a_, b_ in zip(first, again):
            assert np.array_equal(a_, b_)


def _subset_result(res, idx):
    """(scores, runs, offsets) of the pairs at `idx`, compacted."""
    sc, runs, off = res
    parts = [runs[int(off[i]):int(off[i + 1])] for i in idx]
    counts = np.array([len(p) for p in parts], dtype=np.uint64)
    o = np.zeros(len(idx) + 1, dtype=np.uint64)
    np.cumsum(counts, out=o[1:])
    r = np.concatenate(parts).astype(np.uint32) if parts else np.zeros(0, np.uint32)
    return sc[idx], r, o


def _full_size_check(aligner, oracle_lib, synth_lib, name, slot, options=None):
    """A full-size batch in one call, compared with the oracle on every pair
    (scores, offsets and runs byte for byte) and checked for the invariants
    every optimal result has."""
    b = synth_lib.workload(name)
    say(f"case: {name} full size {len(b)} pairs, options {options or 'default'}")
    if options:
        aligner.set_options(**options)
    got = aligner.align(b, PEN, capacity=len(b) * 40 + 1024)
    st = aligner.stats()
    say(f"  stats: {st}")
    check_invariants_vectorized(b, *got, PEN)
    say(f"  oracle on all {len(b)} pairs")
    ref = oracle_all(oracle_lib, b, slot)
    assert_same(got, ref, b, f"{name} all pairs")
    check_sample_cigars(b, *got, PEN, range(0, len(b), len(b) // 400))
    return b, got, st


def test_pairs100_e4_full_size(aligner, oracle_lib, synth_lib):
    """5,000,000 pairs of 100 bp at E = 4 % (the benchmark workload), default
    schedule: every pair against the oracle."""
    _, _, st = _full_size_check(aligner, oracle_lib, synth_lib, "pairs100_e4_5m", 24)
    assert st["short_pairs"] == st["pairs"]


def test_pairs100_e4_full_size_plain_vs_persistent(aligner, oracle_lib, synth_lib, wfa):
    """The same 5,000,000 pairs in the benchmark's launch shape (8 lanes per
    pair, window 32, step cap 16, 256-thread workgroups) as one persistent
    bucketed graph-replayed launch and as the plain per-batch kernel: each
    against the oracle on every pair."""
    shape = dict(window=32, lanes_per_pair=8, step_cap=16, block_threads=256)
    res = {}
    for name, extra in [("persistent", dict(schedule=wfa.WFA_SCHED_PERSISTENT, bucket=1, use_graph=1)),
                        ("plain", dict(schedule=wfa.WFA_SCHED_PLAIN, bucket=-1, use_graph=-1))]:
        _, res[name], st = _full_size_check(aligner, oracle_lib, synth_lib, "pairs100_e4_5m", 24,
                                            {**shape, **extra})
        assert st["short_pairs"] == st["pairs"] and st["lanes_per_pair"] == 8
    for a_, b_ in zip(res["persistent"], res["plain"]):
        assert np.array_equal(a_, b_)


def test_pairs100_e2_full_size(aligner, oracle_lib, synth_lib):
    """5,000,000 pairs of 100 bp at E = 2 %, default schedule: every pair."""
    _full_size_check(aligner, oracle_lib, synth_lib, "pairs100_e2_5m", 16)


def test_pairs100_e2_full_size_benchmarked_launch(aligner, oracle_lib, synth_lib, wfa):
    """The E = 2 % set in the launch the benchmark's autotuner picks for it
    (window 16, 8 lanes per pair, step cap 8, plain kernel, 128-thread
    workgroups): every pair against the oracle; pairs needing more than 8
    steps go through the cascade."""
    _full_size_check(aligner, oracle_lib, synth_lib, "pairs100_e2_5m", 16,
                     dict(schedule=wfa.WFA_SCHED_PLAIN, window=16, lanes_per_pair=8, step_cap=8,
                          block_threads=128, bucket=-1, use_graph=-1))


def test_uneven_full_size(aligner, oracle_lib, synth_lib):
    """2,000,000 uneven pairs (50-300 bp, 0-5 % edits) in one batch: every
    pair against the oracle."""
    _full_size_check(aligner, oracle_lib, synth_lib, "uneven50_300_2m", 80)


def test_long_reads_sample(aligner, oracle_lib, synth_lib, wfa):
    """1-10 kbp pairs with 5-10 % events and indel runs (general kernel,
    wavefront history in the HBM arena): score-only and CIGAR."""
    say("case: long reads 1-10 kbp, score-only 192 pairs")
    b = synth_lib.workload("long1k_10k_100k", 192)
    got = aligner.align(b, PEN, cigar=False)
    assert_same(got, oracle_of(oracle_lib, b, cigar=False), b, "long score")
    say("case: long reads, CIGAR on the 48 shortest of them")
    order = np.argsort(b.p_len, kind="stable")[:48]
    sub = b.subset(order)
    got = aligner.align(sub, PEN, capacity=200_000)
    assert_same(got, oracle_of(oracle_lib, sub), sub, "long cigar")
    check_invariants_vectorized(sub, *got, PEN)
    say("case: long reads, CIGAR on 12 of every length (longest included)")
    order = np.argsort(np.maximum(b.p_len, b.t_len), kind="stable")
    pick = np.unique(np.concatenate([order[::16], order[-2:]]))
    sub = b.subset(pick)
    got = aligner.align(sub, PEN, capacity=400_000)
    assert_same(got, oracle_of(oracle_lib, sub), sub, "long cigar, all lengths")
    check_invariants_vectorized(sub, *got, PEN)


def test_very_long_pair_sequences_outside_lds(aligner, oracle_lib, synth_lib):
    """Pairs of 120-150 kbp (sequences too long for the general kernel's LDS
    copy, so it reads them from HBM): scores and CIGARs bit-exact."""
    say("case: two pairs of 120-150 kbp, score + CIGAR")
    rng = np.random.default_rng(21)
    pairs = []
    for n in (150_000, 120_000):
        p = bytearray(rng.choice(list(b"ACGT"), size=n).astype(np.uint8).tobytes())
        t = bytearray(p)
        for pos in sorted(rng.choice(n - 100, 12, replace=False), reverse=True):
            kind = int(pos) % 3
            if kind == 0:
                t[pos] = b"ACGT"[(b"ACGT".index(t[pos]) + 1) % 4]
            elif kind == 1:
                t[pos:pos] = b"GATTACA"[: 1 + int(pos) % 5]
            else:
                del t[pos:pos + 1 + int(pos) % 4]
        pairs.append((bytes(p), bytes(t)))
    b = synth_lib.from_pairs(pairs)
    got = aligner.align(b, PEN, capacity=10_000)
    assert_same(got, oracle_of(oracle_lib, b), b, "very long")
    check_invariants_vectorized(b, *got, PEN)


def test_history_offset_width_boundary(aligner, oracle_lib, synth_lib):
    """Texts of 65,532-65,537 bases, where the general kernel's CIGAR history
    switches from 16-bit offsets (texts below 65,535 bases, 0xFFFF kept for
    NULL) to 32-bit ones.  Edits sit next to both ends and in between, so the
    backtrace reads history entries at the largest offsets; global and
    ends-free, byte-exact against the oracle."""
    rng = np.random.default_rng(65535)
    pairs = []
    for m in (65532, 65533, 65534, 65535, 65536, 65537):
        t = bytearray(rng.choice(list(b"ACGT"), size=m).astype(np.uint8).tobytes())
        p = bytearray(t)
        spots = sorted({m - 1, m - 3, m - 9, 2, 0, *rng.integers(10, m - 20, 5).tolist()},
                       reverse=True)
        for j, pos in enumerate(spots):
            kind = (j + m) % 3
            if kind == 0:
                p[pos] = b"ACGT"[(b"ACGT".index(p[pos]) + 1) % 4]
            elif kind == 1:
                p[pos:pos] = b"T"
            else:
                del p[pos]
        pairs.append((bytes(p), bytes(t)))
    b = synth_lib.from_pairs(pairs)
    assert sorted(b.t_len.tolist()) == [65532, 65533, 65534, 65535, 65536, 65537]
    for ends in ((0, 0, 0, 0), (3, 4, 5, 2)):
        say(f"case: texts of 65532-65537 bases, ends {ends}, score + CIGAR")
        aligner.set_ends_free(*ends)
        try:
            got = aligner.align(b, PEN, capacity=10_000)
        finally:
            aligner.set_ends_free()
        ref = oracle_lib.align_batch(b, PEN, cigar=True, threads=8, ends=ends)
        assert_same(got, ref, b, f"history width boundary, ends {ends}")
        if ends == (0, 0, 0, 0):
            check_invariants_vectorized(b, *got, PEN)


def test_capacity_error_then_copy(aligner, oracle_lib, synth_lib, wfa):
    """A too-small CIGAR buffer returns WFA_E_CAPACITY with the needed size;
    wfa_copy_last_cigars then delivers the same runs."""
    say("case: capacity error path")
    b = synth_lib.workload("pairs100_e4_5m", 2000, first=77)
    got = aligner.align(b, PEN, capacity=10)  # the wrapper handles E_CAPACITY
    assert aligner.last_needed() == len(got[1])
    assert_same(got, oracle_of(oracle_lib, b), b, "capacity")


def test_alphabet_error(aligner, synth_lib, wfa):
    say("case: non-ACGT byte")
    pairs = [(b"ACGT", b"ACGT"), (b"ACGTACGT", b"ACGNACGT"), (b"acgt", b"ACGT")]
    b = synth_lib.from_pairs(pairs)
    with pytest.raises(wfa.WFAError) as ei:
        aligner.align(b, PEN)
    assert ei.value.status == wfa.WFA_E_ALPHABET and ei.value.bad == 1


def test_too_long_rejected(aligner, wfa):
    """A descriptor over the length limit is rejected before any byte is read."""
    import torch

    say("case: length over WFA_MAX_LENGTH")
    pairs = wfa.pairs_array(np.zeros(3, np.uint64), np.array([4, 4, wfa.WFA_MAX_LENGTH + 1], np.uint32),
                            np.zeros(3, np.uint64), np.array([4, 4, 4], np.uint32))
    dev = torch.from_numpy(pairs.view(np.uint8).copy()).cuda()
    seq = torch.zeros(64, dtype=torch.uint8, device="cuda")
    scores, runs, offsets = aligner.alloc_outputs(3, 100)
    with pytest.raises(wfa.WFAError) as ei:
        aligner.align_device(seq, seq, dev, 3, scores, runs, offsets)
    assert ei.value.status == wfa.WFA_E_TOO_LONG and ei.value.bad == 2


def test_packed_input_and_pack_api(aligner, oracle_lib, synth_lib, wfa):
    """PACKED2 input built with the oracle's plain packer gives the same
    results as ASCII input; wfa_pack2bit reproduces the plain packer."""
    import ctypes

    import torch

    say("case: PACKED2 input path and wfa_pack2bit")
    b = synth_lib.workload("uneven50_300_2m", 3000, first=31)
    n = len(b)
    pw, tw, pst, tst = [], [], [], []
    off_p = off_t = 0
    for i in range(n):
        p, t = b.pair(i)
        wp_, wt_ = oracle_lib.pack2bit(p), oracle_lib.pack2bit(t)
        pst.append(off_p)
        tst.append(off_t)
        pw.append(wp_)
        tw.append(wt_)
        off_p += len(wp_)
        off_t += len(wt_)
    pwords = np.concatenate(pw + [np.zeros(1, np.uint64)])
    twords = np.concatenate(tw + [np.zeros(1, np.uint64)])
    pairs = wfa.pairs_array(np.array(pst, np.uint64), b.p_len, np.array(tst, np.uint64), b.t_len)
    dp = torch.from_numpy(pwords.view(np.uint8).copy()).cuda()
    dt = torch.from_numpy(twords.view(np.uint8).copy()).cuda()
    dpairs = torch.from_numpy(pairs.view(np.uint8).copy()).cuda()
    scores, runs, offsets = aligner.alloc_outputs(n, n * 60)
    need = aligner.align_device(dp, dt, dpairs, n, scores, runs, offsets, encoding=wfa.WFA_PACKED2)
    got = (scores.cpu().numpy(), runs[:need].cpu().numpy().view(np.uint32),
           offsets.cpu().numpy().view(np.uint64))
    assert_same(got, oracle_of(oracle_lib, b), b, "packed2")

    # wfa_pack2bit on the pattern side
    ascii = torch.from_numpy(b.patterns.copy()).cuda()
    starts = torch.from_numpy(b.p_off.view(np.int64).copy()).cuda()
    lens = torch.from_numpy(b.p_len.view(np.int32).copy()).cuda()
    words = torch.zeros(len(pwords) + 8, dtype=torch.int64, device="cuda")
    ws = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    total = ctypes.c_size_t(0)
    bad = ctypes.c_int64(0)
    rc = wfa.wfa_pack2bit(aligner.ctx, ascii.data_ptr(), starts.data_ptr(), lens.data_ptr(), n,
                          words.data_ptr(), words.numel(), ws.data_ptr(), ctypes.byref(total),
                          ctypes.byref(bad), None)
    assert rc == wfa.WFA_OK and bad.value == -1
    assert total.value == len(pwords) - 1
    assert np.array_equal(words[: total.value].cpu().numpy().view(np.uint64), pwords[:-1])
    assert np.array_equal(ws[:n].cpu().numpy(), np.array(pst, np.int64))


def test_autotuner_identical_and_cached(aligner, oracle_lib, synth_lib, tmp_path, wfa):
    """The autotuner checks every candidate gives the same bytes, applies the
    fastest, and reuses its JSON cache entry for the same workload class."""
    say("case: autotuner on uneven 50-300 bp, 40k pairs")
    b = synth_lib.workload("uneven50_300_2m", 40_000, first=4242)
    n = len(b)
    pat, txt, pairs = aligner.to_device(b)
    cache = str(tmp_path / "tune.json")
    chosen = aligner.autotune(pat, txt, pairs, n, PEN, True, sample_pairs=20_000, cache_path=cache)
    say(f"  chosen: {chosen}")
    import json

    data = json.load(open(cache))
    assert len(data) == 1 and "gfx950" in next(iter(data))
    again = aligner.autotune(pat, txt, pairs, n, PEN, True, sample_pairs=20_000, cache_path=cache)
    assert again == chosen
    aligner.set_options(**chosen)
    got = aligner.align(b, PEN)
    assert_same(got, oracle_of(oracle_lib, b), b, "autotuned")
