"""Calls that reuse the same device buffers with new contents.

A call whose buffers, sizes, packed input and settings match the previous
call's starts that call's whole-pass graph before the batch facts are back,
and keeps its results only if the facts lead to the same plan.  These tests
change the batch in place between calls -- same plan with other pairs, a
plan change (a 300-base pair among 100 bp reads), and back -- and compare
every call with the oracle, through the C ABI."""
import numpy as np
import pytest

from gpu_util import assert_same, say

pytestmark = pytest.mark.gpu

PEN = (4, 6, 2)
N = 3000


def _batches(synth_lib):
    a = synth_lib.workload("pairs100_e4_5m", N, first=17)
    b = synth_lib.workload("pairs100_e2_5m", N, first=4242)
    long_pair = synth_lib.workload("uneven50_300_2m", 400, first=3)
    j = int(np.argmax(np.maximum(long_pair.p_len, long_pair.t_len)))
    c = synth_lib.from_pairs([a.pair(i) for i in range(N - 1)] + [long_pair.pair(j)])
    d = synth_lib.workload("uneven50_300_2m", N, first=999)
    e = synth_lib.workload("pairs100_e4_5m", N, first=77_777)
    return [("E=4 %", a), ("E=2 %, same plan", b), ("a 300-base pair: another plan", c),
            ("uneven 50-300 bp", d), ("E=4 % again", e)]


@pytest.mark.parametrize("cigar", [True, False])
def test_same_buffers_new_contents(oracle_lib, synth_lib, cigar):
    import torch

    import paper_2204_02085_amd as wfa

    al = wfa.Aligner(0)
    try:
        words = 64 * N  # room for 2-bit words of up to 2048 bases per pair
        P = torch.zeros(words, dtype=torch.int64, device="cuda")
        T = torch.zeros(words, dtype=torch.int64, device="cuda")
        D = torch.zeros(24 * N, dtype=torch.uint8, device="cuda")
        cap = 200 * N
        scores, runs, offsets = al.alloc_outputs(N, cap, cigar)
        for label, b in _batches(synth_lib):
            assert len(b) == N
            say(f"case: reused buffers, {label}, cigar={cigar}")
            pw, tw, pairs = al.to_device_packed(b)
            P[: pw.numel()].copy_(pw)
            T[: tw.numel()].copy_(tw)
            D.copy_(pairs)
            scores.fill_(-7)
            if cigar:
                runs.fill_(-7)
                offsets.fill_(-7)
            needed = al.align_device(P, T, D, N, scores, runs, offsets, PEN, cigar,
                                     wfa.WFA_PACKED2)
            torch.cuda.synchronize()
            ref = oracle_lib.align_batch(b, PEN, cigar=cigar, threads=8)
            got = (scores.cpu().numpy(),
                   runs[:needed].cpu().numpy().view(np.uint32) if cigar else None,
                   offsets.cpu().numpy().view(np.uint64) if cigar else None)
            assert_same(got, ref, b, f"reused buffers, {label}")
    finally:
        al.close()
