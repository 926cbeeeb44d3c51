"""The device exclusive scan behind CIGAR offsets, word starts and the
general kernel's job offsets, through wfa_pack2bit (whose word starts are
the exclusive scan of ceil(length / 32)): every start and the total against
numpy's cumulative sum, for counts on both sides of the one-block form's
limit (8 tiles of 2048), of tile edges and of the 8192 tiles up to which
each block sums the earlier tiles' totals itself, with a ragged last tile."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def aligner():
    import paper_2204_02085_amd as wfa

    al = wfa.Aligner(0)
    yield al
    al.close()


@pytest.mark.parametrize("n", [1, 2047, 2048, 2049, 16383, 16384, 16385, 18432, 20481, 300_001,
                               17_000_001])
def test_word_starts(aligner, n):
    import torch

    say(f"case: scan of {n} word counts")
    rng = np.random.default_rng(n)
    if n > 1_000_000:  # past 8192 tiles (the tile totals scanned by a pass of their own)
        lens = rng.choice(np.array([0, 1, 33, 70], np.int32), n, p=[0.8, 0.1, 0.06, 0.04])
    else:
        lens = rng.integers(0, 301, n).astype(np.int32)
    lens[rng.integers(0, n, max(1, n // 50))] = 0  # empty sequences scan as 0 words
    ascii = np.full(int(lens.sum()) + 1, ord("A"), np.uint8)
    starts = np.zeros(n, np.int64)
    starts[1:] = np.cumsum(lens[:-1], dtype=np.int64)
    _, ws = aligner.pack2bit(torch.from_numpy(ascii).cuda(), torch.from_numpy(starts).cuda(),
                             torch.from_numpy(lens).cuda())
    torch.cuda.synchronize()
    want = np.zeros(n + 1, np.int64)
    want[1:] = np.cumsum((lens.astype(np.int64) + 31) // 32)
    got = ws.cpu().numpy()
    assert np.array_equal(got, want)  # the starts and, at [n], the total
