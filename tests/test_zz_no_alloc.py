"""The allocation-free entry point (wfa_align_batch_noalloc) against
wfa_align_batch on the same inputs: two calls in a row, the second with a
smaller batch, byte for byte (and the oracle on the first)."""
import ctypes

import numpy as np
import pytest

from gpu_util import assert_same, say

pytestmark = pytest.mark.gpu
PEN = (4, 6, 2)


def _run(wfa, fn, ctx, dev, n, mode):
    import torch

    pat, txt, pairs, scores, runs, offsets = dev
    needed = ctypes.c_size_t(0)
    bad = ctypes.c_int64(-1)
    cigar = mode == wfa.WFA_CIGAR
    scores.fill_(-9)
    if cigar:
        runs.fill_(-9)
        offsets.fill_(-9)
    args = [ctx, pat.data_ptr(), txt.data_ptr(), pairs.data_ptr(), n, wfa.WFA_ASCII]
    if fn is wfa.wfa_align_batch:
        args.append(wfa.WFA_DEVICE)
    args += [wfa.wfa_penalties(*PEN), mode, scores.data_ptr(),
             runs.data_ptr() if cigar else None, runs.numel() if cigar else 0,
             offsets.data_ptr() if cigar else None, ctypes.byref(needed), ctypes.byref(bad), None]
    rc = fn(*args)
    torch.cuda.synchronize()
    assert rc == wfa.WFA_OK, (fn.__name__, rc, bad.value)
    sc = scores.cpu().numpy().copy()
    if not cigar:
        return sc, None, None
    return (sc, runs[: needed.value].cpu().numpy().view(np.uint32).copy(),
            offsets.cpu().numpy().view(np.uint64).copy())


def _long_pairs(synth_lib, k):
    """k pairs of 1-2 kbp at 5-10 % events (general kernel)."""
    lb = synth_lib.workload("long1k_10k_100k", 400)
    idx = np.nonzero(np.maximum(lb.p_len, lb.t_len) < 2000)[0][:k]
    return [lb.pair(int(i)) for i in idx]


def _device(al, b, cap):
    pat, txt, pairs = al.to_device(b)
    return (pat, txt, pairs, *al.alloc_outputs(len(b), cap))


@pytest.mark.parametrize("mode", ["cigar", "score"])
def test_noalloc_equals_align_batch(oracle_lib, synth_lib, mode):
    import paper_2204_02085_amd as wfa

    m = wfa.WFA_CIGAR if mode == "cigar" else wfa.WFA_SCORE
    al = wfa.Aligner(0)
    try:
        # first call: 100 bp pairs at E = 4 % and uneven 50-300 bp pairs (some
        # go through the cascade) plus a few 1-2 kbp pairs (general kernel,
        # arena carved from the scratch array); second call: fewer pairs
        e4 = synth_lib.workload("pairs100_e4_5m", 30_000)
        un = synth_lib.workload("uneven50_300_2m", 8000, first=50)
        big = synth_lib.from_pairs([e4.pair(i) for i in range(len(e4))]
                                   + [un.pair(i) for i in range(len(un))]
                                   + _long_pairs(synth_lib, 6))
        small = synth_lib.workload("uneven50_300_2m", 3000, first=123_456)
        for label, b in (("first", big), ("second", small)):
            say(f"case: noalloc {mode}, {label} call, {len(b)} pairs")
            dev = _device(al, b, len(b) * 60 + 4096)
            ref_entry = _run(wfa, wfa.wfa_align_batch, al.ctx, dev, len(b), m)
            got = _run(wfa, wfa.wfa_align_batch_noalloc, al.ctx, dev, len(b), m)
            for a_, b_ in zip(got, ref_entry):
                if a_ is not None:
                    assert np.array_equal(a_, b_), label
            if label == "first":
                ref = oracle_lib.align_batch(b, PEN, cigar=mode == "cigar", threads=8)
                assert_same(got, ref, b, f"noalloc {label}")
    finally:
        al.close()


def test_noalloc_rejects_over_the_limit(synth_lib):
    import paper_2204_02085_amd as wfa

    say("case: noalloc over the pair limit")
    al = wfa.Aligner(0)
    try:
        n = wfa.WFA_NOALLOC_MAX_PAIRS + 1
        b = synth_lib.workload("pairs100_e2_5m", n)
        dev = _device(al, b, 16)
        pat, txt, pairs, scores, runs, offsets = dev
        scores.fill_(-9)
        needed = ctypes.c_size_t(0)
        bad = ctypes.c_int64(0)
        rc = wfa.wfa_align_batch_noalloc(al.ctx, pat.data_ptr(), txt.data_ptr(), pairs.data_ptr(),
                                         n, wfa.WFA_ASCII, wfa.wfa_penalties(*PEN), wfa.WFA_SCORE,
                                         scores.data_ptr(), None, 0, None, ctypes.byref(needed),
                                         ctypes.byref(bad), None)
        assert rc == wfa.WFA_E_INVAL and bad.value == -1
        assert (scores.cpu().numpy() == -9).all()
    finally:
        al.close()
