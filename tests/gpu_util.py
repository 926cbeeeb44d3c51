"""Helpers shared by the GPU parity tests (no alignment arithmetic here)."""
from __future__ import annotations

import sys

import numpy as np

import brute


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def runs_of(runs: np.ndarray, offsets: np.ndarray, i: int) -> np.ndarray:
    return runs[int(offsets[i]):int(offsets[i + 1])]


def assert_same(gpu, ref, batch=None, label=""):
    """Element-by-element equality of (scores, runs, offsets) with the oracle."""
    sc, runs, off = gpu
    if not np.array_equal(sc, ref.scores):
        bad = np.nonzero(sc != ref.scores)[0]
        i = int(bad[0])
        extra = f" pair {batch.pair(i)}" if batch is not None and len(batch.pair(i)[0]) < 400 else ""
        raise AssertionError(f"{label}: {bad.size} score mismatches; first at {i}: "
                             f"gpu {sc[i]} oracle {ref.scores[i]}{extra}")
    if runs is None:
        return
    if not np.array_equal(off, ref.offsets):
        bad = np.nonzero(off != ref.offsets)[0]
        i = max(int(bad[0]) - 1, 0)
        raise AssertionError(f"{label}: offsets differ from pair {i}: gpu "
                             f"{runs_of(runs, off, i)} oracle {runs_of(ref.runs, ref.offsets, i)}")
    if not np.array_equal(runs, ref.runs):
        j = int(np.nonzero(runs != ref.runs)[0][0])
        i = int(np.searchsorted(off, j, side="right") - 1)
        raise AssertionError(f"{label}: runs differ at pair {i}: gpu {runs_of(runs, off, i)} "
                             f"oracle {runs_of(ref.runs, ref.offsets, i)}")


def check_invariants_vectorized(batch, sc, runs, off, pen):
    """Properties every optimal-alignment result has, checked for all pairs.

    Run lengths are positive, neighbouring runs of a pair differ, the runs
    consume exactly n pattern and m text bases, and the gap-affine cost of the
    runs equals the reported score.
    """
    x, o, e = pen
    N = len(batch)
    counts = np.diff(off.astype(np.int64))
    assert (counts >= 0).all()
    assert int(off[-1]) == runs.size
    ops = (runs & 15).astype(np.int64)
    lens = (runs >> 4).astype(np.int64)
    assert (ops < 4).all() and (lens > 0).all()
    pid = np.repeat(np.arange(N), counts)
    same = (pid[1:] == pid[:-1]) & (ops[1:] == ops[:-1])
    assert not same.any(), "neighbouring runs with the same op"
    used_p = np.bincount(pid, weights=lens * (ops != 2), minlength=N)
    used_t = np.bincount(pid, weights=lens * (ops != 3), minlength=N)
    assert np.array_equal(used_p.astype(np.int64), batch.p_len.astype(np.int64))
    assert np.array_equal(used_t.astype(np.int64), batch.t_len.astype(np.int64))
    cost = np.where(ops == 1, x * lens, 0) + np.where(ops >= 2, o + e * lens, 0)
    total = np.bincount(pid, weights=cost, minlength=N).astype(np.int64)
    assert np.array_equal(total, sc.astype(np.int64)), "runs do not re-score to the score"


def check_sample_cigars(batch, sc, runs, off, pen, idx):
    """Full CIGAR validity (M/X against the bases) on sampled pairs."""
    for i in idx:
        p, t = batch.pair(int(i))
        assert brute.check_cigar(p, t, runs_of(runs, off, int(i)), *pen) == int(sc[int(i)])
