"""A seeded sweep over the library's configuration space, each case checked
byte for byte against the oracle: penalties (including scaled gap
extensions above one step), global and ends-free alignment, short-kernel
shapes, schedules, step caps and the cascade, on pairs of 0-400 bases that
mix related and unrelated sequences and the lengths where offsets switch
from 8 to 16 bits."""
import numpy as np
import pytest

from gpu_util import assert_same, say

pytestmark = pytest.mark.gpu

PENALTIES = [(4, 6, 2), (1, 0, 1), (2, 3, 1), (3, 1, 4), (4, 6, 4), (5, 2, 3), (6, 4, 2)]
SHAPES = [(16, 8), (24, 8), (32, 8), (32, 16), (48, 16), (64, 16), (64, 32), (128, 64),
          (256, 64), (0, 0)]
SCHEDULES = ["AUTO", "PLAIN", "PERSISTENT", "GENERAL"]


@pytest.fixture(scope="module")
def wfa():
    import paper_2204_02085_amd as w

    return w


@pytest.fixture(scope="module")
def aligner(wfa):
    al = wfa.Aligner(0)
    yield al
    al.close()


def make_pairs(rng, count):
    """Related pairs (a few percent to a third of edits), unrelated pairs,
    and pairs whose lengths sit at 0, 1, 127, 128, 255 and 256 bases."""
    out = []
    for i in range(count):
        kind = rng.integers(0, 10)
        if kind < 2:
            n = int(rng.choice([0, 1, 127, 128, 255, 256]))
        else:
            n = int(rng.integers(0, 401))
        p = rng.choice(list(b"ACGT"), n).astype(np.uint8)
        if kind == 9:  # unrelated
            m = int(rng.integers(0, 401))
            t = rng.choice(list(b"ACGT"), m).astype(np.uint8)
        else:
            t = list(p)
            rate = float(rng.choice([0.0, 0.02, 0.05, 0.1, 0.3]))
            for _ in range(int(rng.binomial(max(n, 1), rate))):
                op = int(rng.integers(0, 3))
                pos = int(rng.integers(0, len(t) + 1))
                b = int(rng.choice(list(b"ACGT")))
                if op == 0 and pos < len(t):
                    t[pos] = b
                elif op == 1:
                    t.insert(pos, b)
                elif pos < len(t):
                    del t[pos]
            t = np.array(t, np.uint8)
        out.append((p.tobytes(), t.tobytes()))
    return out


@pytest.mark.parametrize("seed", range(100))
def test_sweep(aligner, oracle_lib, synth_lib, wfa, seed):
    rng = np.random.default_rng(1000 + seed)
    pen = PENALTIES[seed % len(PENALTIES)]
    window, lanes = SHAPES[int(rng.integers(0, len(SHAPES)))]
    sched = SCHEDULES[int(rng.integers(0, len(SCHEDULES)))]
    ends = (0, 0, 0, 0) if seed % 2 == 0 else tuple(int(v) for v in rng.integers(0, 40, 4))
    cascade = int(rng.choice([0, -1, 128]))
    cap = int(rng.choice([0, 0, 6, 12, 24]))
    bucket = int(rng.choice([0, -1]))
    cigar = seed % 3 != 2
    say(f"case: sweep seed {seed}: pen {pen} shape W{window} G{lanes} {sched} ends {ends} "
        f"cascade {cascade} cap {cap} bucket {bucket} cigar {cigar}")
    b = synth_lib.from_pairs(make_pairs(rng, 1200))
    aligner.set_ends_free(*ends)
    aligner.set_options(window=window, lanes_per_pair=lanes,
                        schedule=getattr(wfa, "WFA_SCHED_" + sched), cascade_window=cascade,
                        step_cap=cap, bucket=bucket)
    try:
        got = aligner.align(b, pen, cigar=cigar)
        ref = oracle_lib.align_batch(b, pen, cigar=cigar, threads=8, ends=ends, slot=1024)
        if cigar:
            assert_same(got, ref, b, f"sweep {seed}")
        else:
            assert np.array_equal(got[0], ref.scores)
    finally:
        aligner.set_options()
        aligner.set_ends_free()
