"""GPU parity of host-memory batches, which run as a chunk pipeline (inputs
of chunk k+1 and results of chunk k-1 move while chunk k aligns).

Every case compares scores and CIGAR runs byte for byte with the CPU oracle,
with chunk sizes that leave a ragged last chunk, page-locked and pageable
buffers, a descriptor order that makes the first chunk reach the end of the
sequence buffers, runs that outgrow the device run buffer mid-batch, and the
error paths.
"""
import ctypes
import dataclasses

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


def oracle_of(oracle_lib, batch, pen=PEN, cigar=True):
    return oracle_lib.align_batch(batch, pen, cigar=cigar, threads=8)


@pytest.mark.parametrize("pinned", [False, True])
def test_chunks_ragged_tail(aligner, oracle_lib, synth_lib, wfa, pinned):
    """5,000 pairs in chunks of 700 (8 chunks, the last one of 100)."""
    say(f"case: host pipeline, 5000 pairs, chunks of 700, pinned={pinned}")
    b = synth_lib.workload("pairs100_e4_5m", 5000, first=4242)
    if pinned:
        b.patterns = wfa.host_copy(b.patterns)
        b.texts = wfa.host_copy(b.texts)
    aligner.set_options(host_chunk_pairs=700)
    got = aligner.align_host(b, PEN, pinned=pinned)
    st = aligner.stats()
    assert st["host_chunks"] == 8 and st["pairs"] == 5000
    assert st["cigar_runs"] == len(got[1])
    assert_same(got, oracle_of(oracle_lib, b), b, f"host chunks pinned={pinned}")


def test_chunks_score_only_uneven(aligner, oracle_lib, synth_lib):
    say("case: host pipeline, score only, uneven 50-300 bp, chunks of 333")
    b = synth_lib.workload("uneven50_300_2m", 4000, first=99)
    aligner.set_options(host_chunk_pairs=333)
    sc, _, _ = aligner.align_host(b, PEN, cigar=False)
    ref = oracle_of(oracle_lib, b, cigar=False)
    assert np.array_equal(sc, ref.scores)
    assert aligner.stats()["host_chunks"] == 13


def test_first_chunk_reaches_buffer_end(aligner, oracle_lib, synth_lib):
    """Descriptors in reverse order: the first chunk needs the last bytes of
    both sequence buffers, later chunks need nothing new."""
    say("case: host pipeline, reversed descriptors, chunks of 512")
    b = synth_lib.workload("pairs100_e2_5m", 3000, first=5)
    r = slice(None, None, -1)
    b.p_off, b.p_len, b.t_off, b.t_len = (b.p_off[r].copy(), b.p_len[r].copy(),
                                          b.t_off[r].copy(), b.t_len[r].copy())
    aligner.set_options(host_chunk_pairs=512)
    got = aligner.align_host(b, PEN)
    assert_same(got, oracle_of(oracle_lib, b), b, "reversed")


def test_runs_outgrow_device_buffer(aligner, oracle_lib, synth_lib):
    """Unrelated 100-200 bp pairs (dozens of runs each, more than the first
    estimate of 16 per pair) in chunks of 400: the run buffer grows inside a
    chunk and between chunks while earlier chunks' runs are in flight."""
    say("case: host pipeline, unrelated pairs, runs outgrow the buffer")
    rng = np.random.default_rng(2024)
    pairs = []
    for _ in range(3000):
        n, m = int(rng.integers(100, 201)), int(rng.integers(100, 201))
        pairs.append((bytes(rng.choice(list(b"ACGT"), size=n).astype(np.uint8)),
                      bytes(rng.choice(list(b"ACGT"), size=m).astype(np.uint8))))
    b = synth_lib.from_pairs(pairs)
    aligner.set_options(host_chunk_pairs=400)
    got = aligner.align_host(b, PEN, capacity=3000 * 400)
    assert len(got[1]) > 3000 * 20
    assert_same(got, oracle_of(oracle_lib, b), b, "unrelated")


def test_capacity_error_then_copy(aligner, oracle_lib, synth_lib):
    """Too few runs of room in host memory: WFA_E_CAPACITY after scores and
    offsets, then wfa_copy_last_cigars delivers every run."""
    say("case: host pipeline, capacity error, chunks of 600")
    b = synth_lib.workload("pairs100_e4_5m", 3000, first=321)
    aligner.set_options(host_chunk_pairs=600)
    got = aligner.align_host(b, PEN, capacity=5000)
    assert aligner.last_needed() == len(got[1]) > 5000
    assert_same(got, oracle_of(oracle_lib, b), b, "host capacity")


def test_packed_host_input(aligner, oracle_lib, synth_lib, wfa):
    """2-bit words in page-locked host memory, chunks of 256."""
    say("case: host pipeline, PACKED2 input, chunks of 256")
    b = synth_lib.workload("uneven50_300_2m", 2000, first=17)
    n = len(b)
    pw, tw, pst, tst = [], [], [], []
    off_p = off_t = 0
    for i in range(n):
        p, t = b.pair(i)
        wp_, wt_ = oracle_lib.pack2bit(p), oracle_lib.pack2bit(t)
        pst.append(off_p)
        tst.append(off_t)
        pw.append(wp_)
        tw.append(wt_)
        off_p += len(wp_)
        off_t += len(wt_)
    pwords = wfa.host_copy(np.concatenate(pw + [np.zeros(1, np.uint64)]))
    twords = wfa.host_copy(np.concatenate(tw + [np.zeros(1, np.uint64)]))

    class Words:
        p_off = np.array(pst, np.uint64)
        t_off = np.array(tst, np.uint64)
        p_len = b.p_len
        t_len = b.t_len

    aligner.set_options(host_chunk_pairs=256)
    got = aligner.align_host(Words, PEN, encoding=wfa.WFA_PACKED2, patterns=pwords, texts=twords,
                             pinned=True)
    assert aligner.stats()["host_chunks"] == 8
    assert_same(got, oracle_of(oracle_lib, b), b, "packed host")


def test_alphabet_error_in_later_chunk(aligner, synth_lib, wfa):
    say("case: host pipeline, non-ACGT byte in the fourth chunk")
    b = synth_lib.workload("pairs100_e4_5m", 2000, first=3)
    bad = 1234
    b.texts = b.texts.copy()
    b.texts[int(b.t_off[bad]) + 7] = ord("N")
    aligner.set_options(host_chunk_pairs=400)
    with pytest.raises(wfa.WFAError) as ei:
        aligner.align_host(b, PEN)
    assert ei.value.status == wfa.WFA_E_ALPHABET and ei.value.bad == bad
    # the context stays usable
    b.texts[int(b.t_off[bad]) + 7] = ord("A")
    aligner.align_host(b, PEN)


def test_too_long_rejected_before_any_copy(aligner, wfa):
    """A descriptor over the length limit is found by the host scan, before
    any byte moves (the buffers here are far shorter than it claims)."""
    say("case: host pipeline, length over WFA_MAX_LENGTH")
    n = 3000
    p_len = np.full(n, 4, np.uint32)
    p_len[2500] = wfa.WFA_MAX_LENGTH + 1
    pairs = wfa.pairs_array(np.zeros(n, np.uint64), p_len, np.zeros(n, np.uint64),
                            np.full(n, 4, np.uint32))
    seq = np.frombuffer(b"ACGTACGT", np.uint8).copy()
    scores = np.zeros(n, np.int32)
    offsets = np.zeros(n + 1, np.uint64)
    runs = np.zeros(100, np.uint32)
    needed, badp = ctypes.c_size_t(0), ctypes.c_int64(0)
    aligner.set_options(host_chunk_pairs=500)
    rc = wfa.wfa_align_batch(aligner.ctx, seq.ctypes.data, seq.ctypes.data, pairs.ctypes.data, n,
                             wfa.WFA_ASCII, wfa.WFA_HOST, wfa.wfa_penalties(*PEN), wfa.WFA_CIGAR,
                             scores.ctypes.data, runs.ctypes.data, 100, offsets.ctypes.data,
                             ctypes.byref(needed), ctypes.byref(badp), None)
    assert rc == wfa.WFA_E_TOO_LONG and badp.value == 2500
    assert not scores.any()


def test_empty_and_single_pair(aligner, oracle_lib, synth_lib):
    say("case: host pipeline, empty batch and one pair")
    e = synth_lib.from_pairs([])
    sc, runs, off = aligner.align_host(e, PEN)
    assert len(sc) == 0 and len(runs) == 0 and off.tolist() == [0]
    one = synth_lib.from_pairs([(b"ACGTTGCA", b"ACGTGCA")])
    got = aligner.align_host(one, PEN)
    assert_same(got, oracle_of(oracle_lib, one), one, "one")


def test_large_pageable_batch_copy_threads(aligner, oracle_lib, synth_lib, wfa):
    """Pageable buffers of about 100 MB in (the size from which helper
    threads fill and empty the staging slots, each 32 MB piece split among
    them): 450,000 pairs of 100 bp in one chunk and in the default chunks,
    then the same sequences from page-locked memory (direct DMA).  Every
    score, offset and run equals the device-memory path's on the same batch,
    and a sample of pairs equals the oracle's."""
    n = 450_000
    b = synth_lib.workload("pairs100_e4_5m", n, first=123_457)
    say(f"case: host pipeline, {n} pairs from pageable memory, device path for reference")
    dev = aligner.align(b, PEN)
    for chunk in (n, 0):
        say(f"case: host pipeline, {n} pageable pairs, host_chunk_pairs={chunk}")
        aligner.set_options(host_chunk_pairs=chunk)
        sc, runs, off = aligner.align_host(b, PEN)
        assert np.array_equal(sc, dev[0])
        assert np.array_equal(off, dev[2])
        assert np.array_equal(runs, dev[1])
        say(f"case: host pipeline, {n} pageable pairs, score only, host_chunk_pairs={chunk}")
        sc2, _, _ = aligner.align_host(b, PEN, cigar=False)
        assert np.array_equal(sc2, dev[0])
    say(f"case: host pipeline, {n} pairs from page-locked memory (direct DMA)")
    aligner.set_options()
    pinned = dataclasses.replace(b, patterns=wfa.host_copy(b.patterns),
                                 texts=wfa.host_copy(b.texts))
    sc, runs, off = aligner.align_host(pinned, PEN, pinned=True)
    assert np.array_equal(sc, dev[0]) and np.array_equal(off, dev[2])
    assert np.array_equal(runs, dev[1])
    rng = np.random.default_rng(8)
    idx = np.unique(np.concatenate([rng.choice(n, 3000, replace=False), [0, n - 1]]))
    sub = b.subset(idx)
    pieces = [dev[1][int(dev[2][i]):int(dev[2][i + 1])] for i in idx]
    sub_off = np.zeros(len(idx) + 1, np.uint64)
    np.cumsum([len(p) for p in pieces], out=sub_off[1:])
    assert_same((dev[0][idx], np.concatenate(pieces).astype(np.uint32), sub_off),
                oracle_of(oracle_lib, sub), sub, "large pageable sample")
