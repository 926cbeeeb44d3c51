"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Scores and CIGAR runs must be byte-identical to the oracle's.  Inputs are
the seeded synthetic workloads (pairs of 100 bp reads at 2 % and 4 % edits,
uneven 50-300 bp pairs, long 1-10 kbp pairs) plus edge cases.
"""
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


def test_pairs100_e2_10k_all(aligner, oracle_lib, synth_lib):
    """10,000 pairs of 100 bp at E = 2 %: every pair bit-exact."""
    say("case: pairs100_e2_10k, all pairs, CIGAR, default schedule")
    b = synth_lib.workload("pairs100_e2_10k")
    got = aligner.align(b, PEN)
    assert_same(got, oracle_of(oracle_lib, b), b, "pairs100_e2_10k")
    check_sample_cigars(b, *got, PEN, range(0, len(b), 50))


@pytest.mark.parametrize("schedule", ["PLAIN", "PERSISTENT", "GENERAL", "AUTO"])
def test_pairs100_e4_schedules(aligner, oracle_lib, synth_lib, wfa, schedule):
    say(f"case: pairs100_e4 20k pairs, schedule {schedule}")
    b = synth_lib.workload("pairs100_e4_5m", 20_000)
    aligner.set_options(schedule=getattr(wfa, "WFA_SCHED_" + schedule))
    got = aligner.align(b, PEN)
    assert_same(got, oracle_of(oracle_lib, b), b, f"e4/{schedule}")


@pytest.mark.parametrize("window", [16, 32, 64, 128, 256])
def test_windows_identical(aligner, oracle_lib, synth_lib, wfa, window):
    """Every short-kernel window gives the oracle's bytes (narrow windows
    hand most pairs to the general kernel)."""
    say(f"case: window {window}")
    b = synth_lib.workload("pairs100_e4_5m", 3000, first=50_000)
    aligner.set_options(window=window, schedule=wfa.WFA_SCHED_PERSISTENT)
    got = aligner.align(b, PEN)
    assert_same(got, oracle_of(oracle_lib, b), b, f"window {window}")


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
