"""Serving on the GPU: requests arriving at Poisson times from several
client threads overlap on the device; each request's results equal the
same pairs aligned alone (and the oracle on a sample)."""
import threading
import time

import numpy as np
import pytest

from gpu_util import assert_same, say

pytestmark = pytest.mark.gpu
PEN = (4, 6, 2)


def test_server_mix_equals_alone(oracle_lib, synth_lib):
    import paper_2204_02085_amd as wfa

    say("case: server, 60 Poisson requests of 1-600 pairs, 3 client threads, 4 streams")
    rng = np.random.default_rng(7)
    reqs, first = [], 0
    for i in range(60):
        k = int(round(2 ** rng.uniform(0, np.log2(600))))
        name = "uneven50_300_2m" if i % 3 else "pairs100_e4_5m"
        reqs.append(synth_lib.workload(name, k, first=first))
        first += k
    reqs.append(synth_lib.workload("serving_mix", 24))  # long reads through the general kernel
    al = wfa.Aligner(0)
    srv = wfa.Server(al, hbm_budget_bytes=8 << 30, streams=4, max_chunk_pairs=4096)
    tickets = [None] * len(reqs)

    def client(idxs, seed):
        r = np.random.default_rng(seed)
        for i in idxs:
            time.sleep(float(r.exponential(0.002)))
            tickets[i] = srv.submit(reqs[i])

    ths = [threading.Thread(target=client, args=(range(j, len(reqs), 3), j)) for j in range(3)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    results = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    say(f"  server stats: {st}")
    assert st["max_reserved_bytes"] <= 8 << 30
    for i, (req, res) in enumerate(zip(reqs, results)):
        assert res["status"] == 0
        alone = al.align(req, PEN, capacity=len(req) * 64 + 1024)
        assert np.array_equal(res["scores"], alone[0]), f"request {i} scores"
        assert np.array_equal(res["offsets"], alone[2]), f"request {i} offsets"
        assert np.array_equal(res["runs"], alone[1]), f"request {i} runs"
    for i in (0, 5, len(reqs) - 1):
        ref = oracle_lib.align_batch(reqs[i], PEN, threads=8)
        assert_same((results[i]["scores"], results[i]["runs"], results[i]["offsets"]), ref, reqs[i],
                    f"request {i}")
    al.close()


def test_server_ends_free(oracle_lib, synth_lib):
    """A server opened on a context with free ends aligns every request with
    them (and keeps them after the context returns to global alignment)."""
    import paper_2204_02085_amd as wfa

    say("case: server with free ends (5, 5, 20, 20), 12 requests")
    ends = (5, 5, 20, 20)
    al = wfa.Aligner(0)
    al.set_ends_free(*ends)
    srv = wfa.Server(al, hbm_budget_bytes=4 << 30, streams=2, max_chunk_pairs=2048)
    al.set_ends_free()
    reqs = [synth_lib.workload("uneven50_300_2m", 50 + 40 * i, first=1000 * i) for i in range(12)]
    tickets = [srv.submit(r) for r in reqs]
    results = [srv.poll(t) for t in tickets]
    srv.close()
    for i, (req, res) in enumerate(zip(reqs, results)):
        assert res["status"] == 0
        ref = oracle_lib.align_batch(req, PEN, threads=8, ends=ends)
        assert_same((res["scores"], res["runs"], res["offsets"]), ref, req, f"request {i}")
    al.close()


def test_servers_in_a_row_take_over_engines(oracle_lib, synth_lib):
    """Servers opened one after another on one context take over the engines
    of closed ones: free ends, budgets and stream counts of the new server
    hold (ends-free, then global with a smaller budget and more streams,
    then global with fewer streams), and every result equals the oracle."""
    import paper_2204_02085_amd as wfa

    al = wfa.Aligner(0)
    reqs = [synth_lib.workload("uneven50_300_2m", 40 + 30 * i, first=500 * i) for i in range(8)]
    reqs.append(synth_lib.workload("serving_mix", 12, first=77))
    plan = [((5, 5, 20, 20), 4 << 30, 2), ((0, 0, 0, 0), 1 << 30, 4), ((0, 0, 0, 0), 8 << 30, 3)]
    for k, (ends, budget, streams) in enumerate(plan):
        say(f"case: server {k} of a row, ends {ends}, budget {budget >> 30} GiB, {streams} streams")
        al.set_ends_free(*ends)
        srv = wfa.Server(al, hbm_budget_bytes=budget, streams=streams, max_chunk_pairs=1024)
        al.set_ends_free()
        tickets = [srv.submit(r) for r in reqs]
        results = [srv.poll(t) for t in tickets]
        st = srv.stats()
        srv.close()
        assert st["max_reserved_bytes"] <= budget
        for i, (req, res) in enumerate(zip(reqs, results)):
            assert res["status"] == 0
            ref = oracle_lib.align_batch(req, PEN, threads=8, ends=ends)
            assert_same((res["scores"], res["runs"], res["offsets"]), ref, req,
                        f"server {k} request {i}")
    al.close()


def test_closing_the_context_closes_its_servers(synth_lib):
    """Closing the Aligner first closes servers still open on it (they hand
    their engines to the context), after their submitted work is done."""
    import paper_2204_02085_amd as wfa

    say("case: Aligner.close with a server still open")
    al = wfa.Aligner(0)
    srv = wfa.Server(al, hbm_budget_bytes=1 << 30, streams=2, max_chunk_pairs=512)
    req = synth_lib.workload("pairs100_e4_5m", 300, first=9)
    t = srv.submit(req)
    res = srv.poll(t)
    assert res["status"] == 0 and len(res["scores"]) == 300
    al.close()
    assert srv.srv is None and al.ctx is None
    srv.close()  # a second close is a no-op


def test_server_large_long_requests(oracle_lib, synth_lib):
    """Requests of the serving configuration's largest kind -- 2,048 to 4,096
    pairs of 5-10 kbp reads at 10 % edits -- mixed with small requests of
    100-10,000 bp: every request's results in the mix equal the same pairs
    aligned alone, and an oracle sample (shortest and longest pair of each
    large request, and the small requests whole) matches byte for byte."""
    import paper_2204_02085_amd as wfa

    big_spec = synth_lib.loguniform_single(5000, 10000, 0.10, 0.10)
    sizes = [("small", 3), ("big", 2048), ("small", 40), ("big", 3000), ("small", 1),
             ("big", 4096), ("small", 200)]
    reqs, first = [], 0
    for kind, k in sizes:
        if kind == "big":
            reqs.append(synth_lib.generate(big_spec, 606, k, first=first))
        else:
            reqs.append(synth_lib.workload("serving_mix", k, first=first))
        first += k
    say(f"case: server, {len(reqs)} requests, {sum(k for _, k in sizes)} pairs "
        f"({sum(k for kind, k in sizes if kind == 'big')} of 5-10 kbp at 10 %), CIGAR")
    al = wfa.Aligner(0)
    srv = wfa.Server(al, hbm_budget_bytes=64 << 30, streams=4, max_chunk_pairs=16384)
    tickets = [srv.submit(r) for r in reqs]
    results = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    say(f"  server stats: {st}")
    for i, (req, res) in enumerate(zip(reqs, results)):
        assert res["status"] == 0, f"request {i} status {res['status']}"
        say(f"  request {i}: {len(req)} pairs alone")
        alone = al.align(req, PEN, capacity=len(req) * 1500 + 1024)
        assert np.array_equal(res["scores"], alone[0]), f"request {i} scores"
        assert np.array_equal(res["offsets"], alone[2]), f"request {i} offsets"
        assert np.array_equal(res["runs"], alone[1]), f"request {i} runs"
    for i, (kind, _) in enumerate(sizes):
        req, res = reqs[i], results[i]
        if kind == "big":
            lens = np.maximum(req.p_len, req.t_len)
            idx = [int(np.argmin(lens)), int(np.argmax(lens))]
        else:
            idx = list(range(len(req)))
        say(f"  oracle on {len(idx)} pairs of request {i}")
        sub = req.subset(idx)
        ref = oracle_lib.align_batch(sub, PEN, threads=8)
        parts = [res["runs"][int(res["offsets"][j]):int(res["offsets"][j + 1])] for j in idx]
        off = np.zeros(len(idx) + 1, np.uint64)
        np.cumsum([len(p) for p in parts], out=off[1:])
        got = (res["scores"][idx], np.concatenate(parts).astype(np.uint32), off)
        assert_same(got, ref, sub, f"request {i} oracle sample")
    al.close()
