"""GPU parity of the cascade: pairs a short-kernel pass hands over run again
in wider short-kernel passes (windows 64, 128, 256) before any reaches the
general kernel.  Every result is compared byte for byte with the oracle."""
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
    aligner.set_ends_free()
    yield
    aligner.set_options()
    aligner.set_ends_free()


@pytest.fixture(scope="module")
def uneven(synth_lib):
    return synth_lib.workload("uneven50_300_2m", 4000, first=777)


@pytest.fixture(scope="module")
def uneven_ref(oracle_lib, uneven):
    return oracle_lib.align_batch(uneven, PEN, cigar=True, threads=8)


@pytest.mark.parametrize("first,cascade", [((32, 8), 0), ((32, 8), 64), ((32, 8), 128),
                                           ((16, 8), 0), ((48, 16), 0), ((64, 32), 0),
                                           ((32, 8), -1)])
def test_cascade_levels(aligner, wfa, uneven, uneven_ref, first, cascade):
    """Uneven 50-300 bp pairs from a narrow first window: the cascade's
    passes finish most of the pairs the first pass hands over, and the
    bytes equal the oracle's whatever the levels."""
    window, lanes = first
    say(f"case: cascade from W{window} G{lanes}, largest window {cascade}")
    aligner.set_options(window=window, lanes_per_pair=lanes, schedule=wfa.WFA_SCHED_PERSISTENT,
                        cascade_window=cascade)
    got = aligner.align(uneven, PEN)
    st = aligner.stats()
    assert_same(got, uneven_ref, uneven, f"cascade W{window} -> {cascade}")
    if cascade == -1:
        assert st["cascade_window"] == 0
    else:
        assert st["cascade_window"] >= 64 and st["requeued"] > 0
        if cascade == 0:
            assert st["general_pairs"] < st["requeued"]
    sc, _, _ = aligner.align(uneven, PEN, cigar=False)
    assert np.array_equal(sc, uneven_ref.scores)


def test_cascade_capacity_then_copy(aligner, wfa, uneven, uneven_ref):
    """Runs of cascade passes (kept in their own slots) come back through
    wfa_copy_last_cigars after WFA_E_CAPACITY."""
    say("case: cascade, capacity error path")
    aligner.set_options(window=32, lanes_per_pair=8, schedule=wfa.WFA_SCHED_PERSISTENT)
    got = aligner.align(uneven, PEN, capacity=100)
    assert aligner.stats()["cascade_window"] >= 64
    assert_same(got, uneven_ref, uneven, "cascade capacity")


def test_cascade_ends_free(aligner, oracle_lib, wfa, uneven):
    say("case: cascade with free ends (6, 3, 4, 9)")
    ends = (6, 3, 4, 9)
    aligner.set_ends_free(*ends)
    aligner.set_options(window=32, lanes_per_pair=8, schedule=wfa.WFA_SCHED_PERSISTENT)
    got = aligner.align(uneven, PEN)
    assert aligner.stats()["cascade_window"] >= 64
    assert_same(got, oracle_lib.align_batch(uneven, PEN, cigar=True, threads=8, ends=ends),
                uneven, "cascade ends-free")


def test_cascade_host_pipeline(aligner, wfa, uneven, uneven_ref):
    say("case: cascade inside the host-memory pipeline, chunks of 900")
    aligner.set_options(window=32, lanes_per_pair=8, schedule=wfa.WFA_SCHED_PERSISTENT,
                        host_chunk_pairs=900)
    got = aligner.align_host(uneven, PEN)
    assert_same(got, uneven_ref, uneven, "cascade host")
