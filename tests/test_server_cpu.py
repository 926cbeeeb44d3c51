"""Serving scheduler on the CPU: the C++ admission / continuous-batching
logic of wfa_server_* driven by an executor that runs the CPU oracle.

Checks: every request's results equal the oracle on that request alone;
admission is first-come first-served; the reserved memory never exceeds the
budget; small requests arriving together share batches; a request larger
than the whole budget still completes; chunking of a large request.
"""
import threading
import time

import numpy as np
import pytest


def oracle_executor(oracle_lib, synth_lib, pen, cigar=True, delay=0.0, log=None):
    def run(b):
        pairs = b["pairs"]
        batch = synth_lib.Batch(b["patterns"], b["texts"], pairs["p_start"].astype(np.uint64),
                                pairs["p_len"].astype(np.uint32), pairs["t_start"].astype(np.uint64),
                                pairs["t_len"].astype(np.uint32))
        if log is not None:
            log.append(len(pairs))
        if delay:
            time.sleep(delay)
        r = oracle_lib.align_batch(batch, pen, cigar=cigar, threads=1)
        return r.scores, r.runs, r.offsets
    return run


def make_requests(synth_lib, rng, count, max_pairs):
    reqs = []
    first = 0
    for _ in range(count):
        k = int(rng.integers(1, max_pairs + 1))
        reqs.append(synth_lib.workload("uneven50_300_2m", k, first=first))
        first += k
    return reqs


@pytest.fixture(scope="module")
def wfa():
    import paper_2204_02085_amd as w

    return w


def check_against_oracle(oracle_lib, req, res, pen, cigar=True):
    ref = oracle_lib.align_batch(req, pen, cigar=cigar, threads=2)
    assert res["status"] == 0
    assert np.array_equal(res["scores"], ref.scores)
    if cigar:
        assert np.array_equal(res["offsets"], ref.offsets)
        assert np.array_equal(res["runs"], ref.runs)


def test_server_results_fifo_and_budget(wfa, oracle_lib, synth_lib):
    pen = (4, 6, 2)
    rng = np.random.default_rng(42)
    reqs = make_requests(synth_lib, rng, 30, 40)
    log = []
    probe = wfa.Server(None, executor=oracle_executor(oracle_lib, synth_lib, pen), streams=1)
    sizes = [probe.estimate_bytes(r) for r in reqs]
    probe.close()
    budget = int(max(sizes) * 2.5)
    srv = wfa.Server(None, hbm_budget_bytes=budget, streams=3, max_chunk_pairs=48,
                     executor=oracle_executor(oracle_lib, synth_lib, pen, delay=0.01, log=log))
    tickets = [None] * len(reqs)

    def client(idxs):
        for i in idxs:
            tickets[i] = srv.submit(reqs[i])
            time.sleep(float(rng.exponential(0.002)))

    # one client submits in order so that ticket order is arrival order
    th = threading.Thread(target=client, args=(range(len(reqs)),))
    th.start()
    th.join()
    results = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    for req, res in zip(reqs, results):
        check_against_oracle(oracle_lib, req, res, pen)
    admits = [r["admit"] for r in results]
    assert all(a <= b + 1e-9 for a, b in zip(admits, admits[1:])), "admission not FIFO"
    assert all(r["submit"] <= r["admit"] <= r["done"] for r in results)
    assert st["max_reserved_bytes"] <= budget
    assert st["completed"] == len(reqs) and st["pairs"] == sum(len(r) for r in reqs)
    assert max(log) <= 48
    # pairs of several requests shared batches
    assert st["batches"] < len(reqs)


def test_server_oversized_request_and_chunks(wfa, oracle_lib, synth_lib):
    pen = (4, 6, 2)
    big = synth_lib.workload("uneven50_300_2m", 300, first=5000)
    log = []
    srv = wfa.Server(None, hbm_budget_bytes=1, streams=2, max_chunk_pairs=64,
                     executor=oracle_executor(oracle_lib, synth_lib, pen, log=log))
    t = srv.submit(big)
    res = srv.poll(t)
    st = srv.stats()
    srv.close()
    check_against_oracle(oracle_lib, big, res, pen)
    # nothing fits a 1-byte budget, so pairs ran one at a time, alone
    assert set(log) == {1}
    assert st["batches"] == len(big)


def test_server_score_mode_and_empty(wfa, oracle_lib, synth_lib):
    pen = (2, 3, 1)
    srv = wfa.Server(None, streams=2, max_chunk_pairs=100, penalties=pen, cigar=False,
                     executor=oracle_executor(oracle_lib, synth_lib, pen, cigar=False))
    empty = synth_lib.from_pairs([])
    reqs = [synth_lib.workload("pairs100_e4_5m", k, first=17 * k) for k in (5, 150, 1)]
    ts = [srv.submit(empty)] + [srv.submit(r) for r in reqs]
    out = [srv.poll(t) for t in ts]
    srv.close()
    assert out[0]["num_pairs"] == 0 and out[0]["status"] == 0
    for req, res in zip(reqs, out[1:]):
        check_against_oracle(oracle_lib, req, res, pen, cigar=False)


def test_server_poll_timeout_and_unknown(wfa, oracle_lib, synth_lib):
    pen = (4, 6, 2)
    gate = threading.Event()

    def slow(b):
        gate.wait(10)
        return oracle_executor(oracle_lib, synth_lib, pen)(b)

    srv = wfa.Server(None, streams=1, executor=slow)
    t = srv.submit(synth_lib.workload("pairs100_e2_10k", 3))
    assert srv.poll(t, timeout_us=1000) is None  # still running
    gate.set()
    assert srv.poll(t)["status"] == 0
    with pytest.raises(wfa.WFAError):
        srv.poll(t + 1000, timeout_us=0)
    srv.close()
