"""GPU tests of the C ABI's argument checks, error statuses and limits.

Every call goes through the library's C entry points (ctypes marshalling
only); results that are returned are compared with the CPU oracle.
"""
import ctypes

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
    yield
    aligner.set_options()


def _call(wfa, ctx, dev, n, pen, mode, capacity=None):
    """wfa_align_batch on device tensors; returns (status, needed, bad)."""
    pat, txt, pairs, scores, runs, offsets = dev
    needed = ctypes.c_size_t(0)
    bad = ctypes.c_int64(-1)
    cigar = mode == wfa.WFA_CIGAR
    cap = (runs.numel() if capacity is None else capacity) if cigar else 0
    rc = wfa.wfa_align_batch(ctx, pat.data_ptr(), txt.data_ptr(), pairs.data_ptr(), n,
                             wfa.WFA_ASCII, wfa.WFA_DEVICE, wfa.wfa_penalties(*pen), mode,
                             scores.data_ptr(), runs.data_ptr() if cigar else None, cap,
                             offsets.data_ptr() if cigar else None, ctypes.byref(needed),
                             ctypes.byref(bad), None)
    import torch

    torch.cuda.synchronize()
    return rc, needed.value, bad.value


@pytest.mark.parametrize("pen", [(0, 6, 2), (4, 6, 0), (4, -1, 2), (-4, 6, 2), (4, 6, -2)])
def test_invalid_penalties_rejected(aligner, synth_lib, wfa, pen):
    """x <= 0, e <= 0 or o < 0 is WFA_E_INVAL, and nothing is written."""
    say(f"case: invalid penalties {pen}")
    b = synth_lib.workload("pairs100_e4_5m", 100)
    pat, txt, pairs = aligner.to_device(b)
    scores, runs, offsets = aligner.alloc_outputs(100, 5000)
    scores.fill_(-77)
    rc, _, bad = _call(wfa, aligner.ctx, (pat, txt, pairs, scores, runs, offsets), 100, pen,
                       wfa.WFA_CIGAR)
    assert rc == wfa.WFA_E_INVAL and bad == -1
    assert (scores.cpu().numpy() == -77).all()


def test_graph_replay_respects_capacity(aligner, oracle_lib, synth_lib, wfa):
    """Graphs replayed for the same buffers, pairs and plan but a different
    CIGAR capacity: a smaller capacity gives WFA_E_CAPACITY and writes no run
    at or past it; a larger one gives the oracle's runs."""
    import torch

    b = synth_lib.workload("pairs100_e4_5m", 20_000, first=31_000)
    n = len(b)
    pat, txt, pairs = aligner.to_device(b)
    scores, runs, offsets = aligner.alloc_outputs(n, n * 40)
    ref = oracle_lib.align_batch(b, PEN, cigar=True, threads=8)
    total = int(ref.offsets[-1])
    small = total // 2
    aligner.set_options(schedule=wfa.WFA_SCHED_PERSISTENT, use_graph=1)
    for order in (("full", "small", "full"), ("small", "full", "small")):
        for what in order:
            say(f"case: graph replay capacity order {order}, now {what}")
            runs.fill_(-5)
            cap = runs.numel() if what == "full" else small
            view = runs if what == "full" else runs[:small]
            rc, needed, _ = _call(wfa, aligner.ctx, (pat, txt, pairs, scores, view, offsets), n,
                                  PEN, wfa.WFA_CIGAR, capacity=cap)
            assert needed == total
            assert aligner.stats()["graph_replayed"] == 1
            r = runs.cpu().numpy().view(np.uint32)
            if what == "small":
                assert rc == wfa.WFA_E_CAPACITY
                assert (r[small:] == np.uint32(0xFFFFFFFB)).all(), "runs written past capacity"
                assert np.array_equal(scores.cpu().numpy(), ref.scores)
            else:
                assert rc == wfa.WFA_OK
                got = (scores.cpu().numpy(), r[:total], offsets.cpu().numpy().view(np.uint64))
                assert_same(got, ref, b, f"capacity order {order}")
    torch.cuda.synchronize()


def test_general_step_limit_gives_up(aligner, oracle_lib, synth_lib, wfa):
    """A general-kernel step limit below a pair's score makes the kernel give
    up on it and exit normally; the call returns WFA_E_LIMIT naming the
    lowest such pair, and every other pair's score is still the oracle's."""
    b = synth_lib.workload("uneven50_300_2m", 400, first=777)
    ref = oracle_lib.align_batch(b, PEN, cigar=False, threads=8)
    limit = 20  # steps of gcd(4, 6, 2) = 2
    over = np.nonzero(ref.scores // 2 > limit)[0]
    assert over.size > 0 and over.size < len(b)
    for cigar in (False, True):
        say(f"case: general kernel step limit {limit}, cigar {cigar}")
        aligner.set_options(schedule=wfa.WFA_SCHED_GENERAL, general_step_limit=limit)
        n = len(b)
        pat, txt, pairs = aligner.to_device(b)
        scores, runs, offsets = aligner.alloc_outputs(n, n * 200)
        mode = wfa.WFA_CIGAR if cigar else wfa.WFA_SCORE
        rc, _, bad = _call(wfa, aligner.ctx, (pat, txt, pairs, scores, runs, offsets), n, PEN, mode)
        assert rc == wfa.WFA_E_LIMIT, wfa.wfa_strerror(rc)
        assert bad == int(over[0])
        sc = scores.cpu().numpy()
        ok = np.ones(n, bool)
        ok[over] = False
        assert (sc[over] == -1).all()
        assert np.array_equal(sc[ok], ref.scores[ok])
    # without the limit the same batch aligns
    aligner.set_options(schedule=wfa.WFA_SCHED_GENERAL)
    got = aligner.align(b, PEN)
    assert_same(got, oracle_lib.align_batch(b, PEN, cigar=True, threads=8), b, "no limit")


def test_general_slice_requeue(aligner, oracle_lib, synth_lib, wfa):
    """CIGAR histories that outgrow a deliberately small first slice are
    re-run with 4x slices (counted in wfa_stats.requeued) and still give the
    oracle's bytes."""
    say("case: general kernel, 16 KiB first slices, long pairs with CIGAR")
    b = synth_lib.workload("long1k_10k_100k", 40, first=300)
    aligner.set_options(schedule=wfa.WFA_SCHED_GENERAL, general_slice_kib=16)
    got = aligner.align(b, PEN, capacity=200_000)
    st = aligner.stats()
    say(f"  stats: {st}")
    assert st["requeued"] > 0 and st["general_pairs"] == len(b)
    assert_same(got, oracle_lib.align_batch(b, PEN, cigar=True, threads=8), b, "requeue")


def test_tiny_budget(wfa, synth_lib, oracle_lib):
    """A context whose budget cannot hold a batch's device workspace returns
    WFA_E_NOMEM (no fault, nothing half-written that is reported as done);
    batches that fit still align on the same context."""
    ctx = ctypes.c_void_p()
    assert wfa.wfa_ctx_create(0, 256 << 10, ctypes.byref(ctx)) == wfa.WFA_OK
    try:
        import torch

        def run(b, mode):
            n = len(b)
            pairs = wfa.pairs_array(b.p_off, b.p_len, b.t_off, b.t_len)
            dev = (torch.from_numpy(b.patterns.copy()).cuda(), torch.from_numpy(b.texts.copy()).cuda(),
                   torch.from_numpy(pairs.view(np.uint8).copy()).cuda(),
                   torch.empty(n, dtype=torch.int32, device="cuda"),
                   torch.empty(n * 60 + 64, dtype=torch.int32, device="cuda"),
                   torch.empty(n + 1, dtype=torch.int64, device="cuda"))
            return _call(wfa, ctx, dev, n, PEN, mode), dev

        say("case: 256 KiB budget, 20k pairs of 100 bp")
        (rc, _, _), _ = run(synth_lib.workload("pairs100_e4_5m", 20_000), wfa.WFA_CIGAR)
        assert rc == wfa.WFA_E_NOMEM
        say("case: 256 KiB budget, one pair of more than 3 kbp (general kernel arena)")
        lb = synth_lib.workload("long1k_10k_100k", 50)
        big = int(np.nonzero(np.minimum(lb.p_len, lb.t_len) > 3000)[0][0])
        (rc, _, _), _ = run(lb.subset([big]), wfa.WFA_CIGAR)
        assert rc == wfa.WFA_E_NOMEM
        say("case: 256 KiB budget, 200 pairs of 100 bp fit")
        b = synth_lib.workload("pairs100_e4_5m", 200)
        (rc, need, _), dev = run(b, wfa.WFA_CIGAR)
        assert rc == wfa.WFA_OK
        got = (dev[3].cpu().numpy(), dev[4][:need].cpu().numpy().view(np.uint32),
               dev[5].cpu().numpy().view(np.uint64))
        assert_same(got, oracle_lib.align_batch(b, PEN, cigar=True, threads=4), b, "tiny budget")
    finally:
        wfa.wfa_ctx_destroy(ctx)


def test_set_options_rejects_bad_values(aligner, wfa):
    for kw in (dict(use_graph=3), dict(bucket=2), dict(general_step_limit=-1),
               dict(general_slice_kib=-1), dict(window=40), dict(lanes_per_pair=12),
               dict(block_threads=96)):
        with pytest.raises(wfa.WFAError) as ei:
            aligner.set_options(**kw)
        assert ei.value.status == wfa.WFA_E_INVAL
