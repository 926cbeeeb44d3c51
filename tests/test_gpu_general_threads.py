"""The general kernel at each workgroup size its launch picks for pairs above
600 bases -- 1024 threads per pair up to 8 pairs per compute unit, 512 up to
24 and 256 beyond -- against the CPU oracle on every pair: scores and CIGAR
runs through the C ABI, full histories and checkpoints, score-only too."""
import numpy as np
import pytest

from gpu_util import assert_same, say

pytestmark = pytest.mark.gpu

PEN = (4, 6, 2)
GENERAL = 3  # WFA_SCHED_GENERAL


@pytest.fixture(scope="module")
def aligner():
    import paper_2204_02085_amd as wfa

    al = wfa.Aligner(0)
    yield al
    al.set_options()
    al.close()


# 256 compute units: 400 pairs -> 2 per CU (1024 threads), 3000 -> 12 (512),
# 7000 -> 28 (256)
@pytest.mark.parametrize("count", [400, 3000, 7000])
def test_workgroup_sizes(aligner, oracle_lib, synth_lib, count):
    b = synth_lib.generate(synth_lib.long_reads(601, 1200, 0.02, 0.08), 4100 + count, count)
    assert int(np.maximum(b.p_len, b.t_len).min()) > 600
    slot = int((b.p_len.astype(np.int64) + b.t_len).max()) + 1
    cap = int((b.p_len.astype(np.int64) + b.t_len).sum()) + 1024
    ref = oracle_lib.align_batch(b, PEN, cigar=True, threads=16, slot=slot)
    for ck in (-1, 128):  # full histories, checkpoints every 128 steps
        say(f"case: {count} pairs of 601-1200 bp on the general kernel, checkpoint {ck}")
        aligner.set_options(schedule=GENERAL, general_checkpoint=ck)
        got = aligner.align(b, PEN, capacity=cap)
        assert_same(got, ref, b, f"{count} pairs, checkpoint {ck}")
        assert aligner.stats()["general_pairs"] == count
    say(f"case: {count} pairs of 601-1200 bp on the general kernel, score only")
    aligner.set_options(schedule=GENERAL)
    got = aligner.align(b, PEN, cigar=False)
    assert np.array_equal(got[0], ref.scores)
