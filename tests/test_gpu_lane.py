"""GPU parity of the one-pair-per-lane kernel (wavefront rows in registers,
unrolled over the cells the (4, 6, 2) recurrences can reach): every result
byte-identical to the oracle, in both step caps, both launch forms and both
modes, including pairs it must hand over (lengths past 127, target diagonals
outside its cells, more steps than its cap)."""
import numpy as np
import pytest

from gpu_util import assert_same, check_invariants_vectorized, say

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


def _mixed_batch(synth_lib, rng):
    """100 bp pairs at E = 4 % and 2 %, and edge pairs: empty, identical,
    one base, short sequences (diagonals off the matrix), unrelated pairs
    (most need more steps than the cap), lengths 126-128, length differences
    beyond the kernel's diagonals."""
    pairs = []
    for name, first in (("pairs100_e4_5m", 7_000), ("pairs100_e2_5m", 3_000)):
        b = synth_lib.workload(name, 6000, first=first)
        pairs += [b.pair(i) for i in range(len(b))]
    pairs += [(b"", b""), (b"", b"ACG"), (b"ACGTA", b""), (b"A", b"A"), (b"A", b"C"),
              (b"AC", b"CA"), (b"ACGT" * 31 + b"AC", b"ACGT" * 31 + b"AC"),
              (b"A" * 127, b"A" * 114), (b"C" * 120, b"C" * 127), (b"G" * 127, b"T" * 127)]
    pairs += synth_lib.random_pairs(rng, 400, 40)
    pairs += synth_lib.random_pairs(rng, 200, 127)
    pairs += synth_lib.random_pairs(rng, 100, 127, related=False)
    # related pairs may have grown past 127 bases by insertions
    pairs = [(p, t) for p, t in pairs if len(p) <= 127 and len(t) <= 127]
    return synth_lib.from_pairs(pairs)


@pytest.mark.parametrize("cap", [8, 16])
@pytest.mark.parametrize("schedule", ["PLAIN", "PERSISTENT"])
@pytest.mark.parametrize("cigar", [True, False])
def test_lane_kernel_matches_oracle(aligner, oracle_lib, synth_lib, wfa, cap, schedule, cigar):
    rng = np.random.default_rng(cap * 7 + (schedule == "PLAIN") + 2 * cigar)
    b = _mixed_batch(synth_lib, rng)
    assert int(max(b.p_len.max(), b.t_len.max())) <= 127
    say(f"case: lane kernel cap {cap}, {schedule}, cigar {cigar}, {len(b)} pairs")
    aligner.set_options(schedule=getattr(wfa, "WFA_SCHED_" + schedule), step_cap=cap,
                        lane_kernel=1, block_threads=256 if cap == 16 else 128)
    got = aligner.align(b, PEN, cigar=cigar, capacity=len(b) * 80)
    st = aligner.stats()
    say(f"  stats: {st}")
    assert st["lane_kernel"] == 1 and st["step_cap"] == cap
    assert st["short_pairs"] + st["general_pairs"] == len(b)
    assert st["requeued"] > 0  # the edge pairs went on to the cascade
    ref = oracle_lib.align_batch(b, PEN, cigar=cigar, threads=8)
    assert_same(got, ref, b, f"lane cap {cap} {schedule} cigar {cigar}")
    if cigar:
        check_invariants_vectorized(b, *got, PEN)


def test_lane_kernel_not_used_past_127(aligner, oracle_lib, synth_lib, wfa):
    """A batch with a 128-base sequence runs on the short kernel instead."""
    b = synth_lib.from_pairs([synth_lib.workload("pairs100_e4_5m", 1).pair(0),
                              (b"ACGT" * 32, b"ACGT" * 31 + b"ACGA")])
    got = aligner.align(b, PEN)
    assert aligner.stats()["lane_kernel"] == 0
    assert_same(got, oracle_lib.align_batch(b, PEN, threads=2), b, "128 bases")


def test_lane_kernel_graph_replays(aligner, oracle_lib, synth_lib, wfa):
    """The lane kernel inside the captured whole-pass graph, replayed with
    eager device work between replays: every replay gives the oracle's bytes."""
    import torch

    b = synth_lib.workload("pairs100_e4_5m", 50_000, first=400_000)
    n = len(b)
    pat, txt, pairs = aligner.to_device(b)
    scores, runs, offsets = aligner.alloc_outputs(n, n * 40)
    ref = oracle_lib.align_batch(b, PEN, threads=8)
    aligner.set_options(schedule=wfa.WFA_SCHED_PERSISTENT, use_graph=1)
    for rep in range(3):
        say(f"case: lane kernel graph replay {rep}")
        scores.fill_(-3)
        runs.fill_(0)
        junk = torch.randn(1 << 20, device=scores.device).sum()
        torch.cuda.synchronize()
        need = aligner.align_device(pat, txt, pairs, n, scores, runs, offsets)
        st = aligner.stats()
        assert st["graph_replayed"] == 1 and st["lane_kernel"] == 1
        got = (scores.cpu().numpy(), runs[:need].cpu().numpy().view(np.uint32),
               offsets.cpu().numpy().view(np.uint64))
        assert_same(got, ref, b, f"replay {rep}")
        del junk
