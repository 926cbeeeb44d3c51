"""Throughput of batched gap-affine WFA alignment on one MI355X.

Workload: 5,000,000 synthetic pairs of 100 bp reads with exactly 4 edits
(E = 4 %; substitutions, insertions and deletions with probability 1/3
each), penalties x=4, o=6, e=2, score + CIGAR.  The paper's experiment
aligns 5 million 100 bp pairs at E = 2 % and 4 % (Results); its read set is
not public, so a seeded generator stands in for it.

One step = one wfa_align_batch call over the whole batch with the inputs
already resident in HBM as 2-bit packed uint64 words (the library's own
packer runs once before timing; `--encoding ascii` times ASCII input, which
adds the packing to every step): (bucketing,) the short-pair kernel, the
general kernel for any pair it hands over, CIGAR offsets and compaction into
the caller's device buffers.  The launch options are picked by the
library's autotuner on a sample of the batch before timing.  The persistent
(bucketed, graph-replayed) and the plain (one launch, no bucketing)
schedules with default knobs are timed on the same bytes and reported
beside it, as is a serving run (p50/p99 latency under Poisson load).

Printed: one JSON line (see the keys below).  `roofline` describes the
dominant kernel (the short-pair alignment kernel); its duration comes from
HIP events the library records around that kernel on the stream it runs on.
`cpu_baseline` times the CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz -> 32-bit integer VALU lane-ops/s
PEAK_INT_OPS = 256 * 4 * 16 * 2.4e9
# Cost models of the algorithm (integer ops, independent of any kernel).
# Primary (the scope table's): ~14 ops per wavefront cell (three state
# updates with their admissibility tests) and ~25 per 32-base extension
# word compare.  Second (itemised): a cell as 5 source reads, 3 candidate
# increments, 5 admissibility tests, 4 maxima, 3 stores = 20 ops; a compare
# as offsets (2), two 2-word window extractions (6), xor (2), trailing-zero
# count (3), clamps to the ends (3), advance (2) = 18 ops.
OPS_PER_CELL, OPS_PER_WINDOW = 14, 25
OPS_PER_CELL_ITEMISED, OPS_PER_WINDOW_ITEMISED = 20, 18
WORKLOAD = "pairs100_e4_5m"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--pairs", type=int, default=5_000_000)
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--encoding", choices=["packed2", "ascii"], default="packed2",
                    help="input encoding resident in HBM")
    ap.add_argument("--mode", choices=["cigar", "score"], default="cigar",
                    help="result mode of the timed workload")
    ap.add_argument("--second-set", default="pairs100_e2_5m",
                    help="the configuration's second set (E = 2 %%), timed the same way after "
                         "the main workload; 'none' or empty: skip")
    ap.add_argument("--other-configs", type=int, default=1,
                    help="also time the uneven (2M pairs, autotuned) and long-read (100k pairs, "
                         "score-only and CIGAR) configurations, and the main workload score-only "
                         "and ends-free (0: skip)")
    ap.add_argument("--host-steps", type=int, default=2,
                    help="calls timed with host ASCII inputs and host outputs (PCIe "
                         "included; 0: skip)")
    ap.add_argument("--tune-sample", type=int, default=0,
                    help="pairs the autotuner times candidates on (0: as many as the timed "
                         "batch): the pairs of the same seeded stream right after the timed "
                         "batch, so tuning never sees the timed inputs")
    ap.add_argument("--options", default="",
                    help="JSON launch options instead of autotuning (profiling runs)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (PMC scale calibration)")
    ap.add_argument("--calib-read-mib", type=int, default=0,
                    help="first sum this many MiB of int32 (a read-only kernel of known bytes, "
                         "PMC read-scale calibration)")
    ap.add_argument("--cpu-pairs", type=int, default=2_000_000,
                    help="oracle sample size for the CPU baseline, about 15 s of CPU time "
                         "on 16 threads (0: skip)")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--serving-requests", type=int, default=200,
                    help="requests of the serving run (0: skip)")
    ap.add_argument("--serving-load", type=float, default=0.75,
                    help="offered load (fraction of the measured saturation rate) whose "
                         "latencies are reported as the serving p50/p99")
    ap.add_argument("--serving-chunk", type=int, default=16384,
                    help="most pairs per batch the server launches (max_chunk_pairs)")
    ap.add_argument("--serving-sweep", default="0.25,0.5",
                    help="further offered loads of the rate sweep, comma-separated ('none': "
                         "only --serving-load)")
    return ap.parse_args()


def log(msg: str):
    """Progress on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_label(st: dict) -> str:
    """Name of the kernel a call's first pass ran (from its statistics)."""
    if st.get("lane_kernel"):
        return f"k_lane<one pair per lane, step cap {st['step_cap']}, cigar>"
    return (f"k_short<window {st['window']}, {st['lanes_per_pair']} lanes per pair, "
            f"step cap {st['step_cap']}, cigar>")


def kernel_source_hash() -> str:
    """Hash of the source of the one-pair-per-lane kernel (the headline's
    dominant kernel)."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2204_02085_amd", "csrc", "k_lane.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def read_profile(kernel_hash: str, label: str) -> dict:
    """Figures of the committed rocprofv3 summary of the headline kernel (HBM
    bytes per launch, VALU issue rate, VALU instructions per pair), if it was
    taken on the current kernel source and the same kernel launch; empty
    otherwise."""
    path = os.path.join(ROOT, "profiles", "k_lane_pairs100_e4_5m.txt")
    if not os.path.exists(path):
        return {}
    vals = {}
    with open(path) as f:
        for line in f:
            if " = " in line and not line.startswith("#"):
                k, v = line.split(" = ", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_hash or vals.get("kernel_label") != label:
        return {}
    out = {}
    for k in ("hbm_bytes_per_launch", "valu_issue_per_cu_cycle", "traffic_over_algorithmic",
              "valu_insts_per_pair"):
        try:
            out[k] = float(vals[k])
        except (KeyError, ValueError):
            pass
    return out


def tune_on_disjoint_sample(al, wfa, synth, workload, n, count, enc, cigar=True):
    """Autotune on `count` pairs of the same seeded stream that follow the
    `n` pairs of the timed batch (never the timed inputs themselves)."""
    import torch

    sample = synth.workload(workload, count, first=n)
    if enc == wfa.WFA_PACKED2:
        sp, st_, sd = al.to_device_packed(sample)
    else:
        sp, st_, sd = al.to_device(sample)
    chosen = al.autotune(sp, st_, sd, len(sample), (4, 6, 2), cigar, encoding=enc,
                         sample_pairs=len(sample))
    del sp, st_, sd
    torch.cuda.synchronize()
    return chosen


def time_schedule(al, dev, n, steps, warmup, options, enc, cigar=True):
    import torch

    al.set_options(**options)
    pat, txt, pairs, scores, runs, offsets = dev
    for _ in range(warmup):
        al.align_device(pat, txt, pairs, n, scores, runs, offsets, (4, 6, 2), cigar, enc)
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        al.align_device(pat, txt, pairs, n, scores, runs, offsets, (4, 6, 2), cigar, enc)
        kernel_ms.append(al.stats()["ms_align"] + al.stats()["ms_general"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = al.stats()
    return (t1 - t0), kernel_ms, st


def host_path_run(al, wfa, batch, steps, options):
    """Whole calls with host memory on both sides: ASCII pairs in host
    buffers, results back in host buffers, through the library's chunk
    pipeline (copies in, alignment and copies out of successive chunks
    overlap).  Timed twice: with pageable numpy buffers and with page-locked
    buffers from wfa_host_alloc.  PCIe is included; this is never the
    headline value."""
    import ctypes

    import numpy as np

    n = len(batch.p_len)
    cap = n * 40 + 1024
    al.set_options(**options)

    ascii_in = (wfa.WFA_ASCII, batch.patterns, batch.texts,
                wfa.pairs_array(batch.p_off, batch.p_len, batch.t_off, batch.t_len))

    def run(pinned, inputs):
        enc = inputs[0]
        empty = wfa.host_empty if pinned else np.empty
        copy = wfa.host_copy if pinned else (lambda a: a)
        pat, txt, pairs = (copy(a) for a in inputs[1:])
        scores = empty(n, np.int32)
        offsets = empty(n + 1, np.uint64)
        runs = empty(cap, np.uint32)
        needed = ctypes.c_size_t(0)
        bad = ctypes.c_int64(-1)

        def call():
            rc = wfa.wfa_align_batch(al.ctx, pat.ctypes.data, txt.ctypes.data, pairs.ctypes.data,
                                     n, enc, wfa.WFA_HOST, wfa.wfa_penalties(4, 6, 2),
                                     wfa.WFA_CIGAR, scores.ctypes.data, runs.ctypes.data, cap,
                                     offsets.ctypes.data, ctypes.byref(needed), ctypes.byref(bad),
                                     None)
            if rc != wfa.WFA_OK:
                raise wfa.WFAError(rc, "wfa_align_batch (host)", bad.value)

        call()
        t0 = time.perf_counter()
        for _ in range(steps):
            call()
        el = time.perf_counter() - t0
        st = al.stats()
        moved = (pat.nbytes + txt.nbytes + pairs.nbytes + scores.nbytes + offsets.nbytes
                 + needed.value * 4)
        return {"pairs_per_s": n * steps / el, "ms_per_call": el / steps * 1e3,
                "chunks": st["host_chunks"], "pcie_gb_per_s": moved * steps / el / 1e9,
                "bytes_moved_per_call": moved}, np.array(scores)

    pageable, scores = run(False, ascii_in)
    pinned, scores2 = run(True, ascii_in)
    # the same pairs as 2-bit words (packed once by the library, then kept in
    # host memory): a quarter of the sequence bytes cross the link
    pw, tw, dpairs = al.to_device_packed(batch)
    packed_in = (wfa.WFA_PACKED2, pw.cpu().numpy(), tw.cpu().numpy(),
                 dpairs.cpu().numpy().view(wfa.PAIR_DTYPE))
    del pw, tw, dpairs
    packed, scores3 = run(True, packed_in)
    if not (np.array_equal(scores, scores2) and np.array_equal(scores, scores3)):
        raise SystemExit("host path: pinned, pageable and packed calls disagree")
    out = {"steps": steps, "input": "ASCII in host memory", "output": "host memory",
           "pageable": pageable, "pinned": pinned, "pinned_packed2_input": packed}
    return out, scores


def serving_run(al, wfa, synth, n_req, load, sweep=(), chunk=16384, seed=11):
    """Poisson requests of 1-4096 pairs (log-uniform), 100-10,000 bp reads
    with 1-10 % edits, CIGAR mode, 64 GiB admission budget, 4 streams.
    First all requests at once (saturation), then Poisson arrivals at each
    offered load of the sweep (a fraction of the saturation request rate,
    `load` among them); latency = done - submit."""
    import threading

    import numpy as np
    import torch

    rng = np.random.default_rng(seed)
    sizes = np.round(2.0 ** rng.uniform(0, 12, n_req)).astype(int)
    reqs, first = [], 0
    for k in sizes:
        reqs.append(synth.workload("serving_mix", int(k), first=first))
        first += int(k)
    total_pairs = int(sizes.sum())

    # one long-lived server for the whole sweep, as a service would run
    srv = wfa.Server(al, hbm_budget_bytes=64 << 30, streams=4, max_chunk_pairs=chunk)

    # requests whose results are compared with the CPU oracle (the six with
    # the fewest bases, so the check stays within seconds)
    import oracle

    bases = [int(r.p_len.sum()) + int(r.t_len.sum()) for r in reqs]
    checked = sorted(range(n_req), key=lambda i: bases[i])[:6]

    def run(gaps, check=False):
        st0 = srv.stats()
        tickets = [None] * n_req

        def client():
            t_next = time.perf_counter()
            for i in range(n_req):
                t_next += gaps[i]
                dt = t_next - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                tickets[i] = srv.submit(reqs[i])

        t0 = time.perf_counter()
        th = threading.Thread(target=client)
        th.start()
        th.join()
        res = [srv.poll(t) for t in tickets]
        t1 = time.perf_counter()
        st = srv.stats()
        for t in tickets:
            srv.release(t)
        bad = [r for r in res if r["status"] != 0]
        if bad:
            codes = sorted({int(r["status"]) for r in bad})
            raise RuntimeError(f"{len(bad)} serving requests failed with status {codes}")
        if check:
            for i in checked:
                ref = oracle.align_batch(reqs[i], (4, 6, 2), cigar=True, threads=8)
                r = res[i]
                if not (np.array_equal(r["scores"], ref.scores)
                        and np.array_equal(r["offsets"], ref.offsets)
                        and np.array_equal(r["runs"], ref.runs)):
                    print(f"bench: serving request {i} differs from the oracle", file=sys.stderr)
                    sys.exit(3)
            log(f"serving parity: requests {checked} equal the oracle byte for byte")
        lat = np.array([r["done"] - r["submit"] for r in res]) * 1e3
        wait = np.array([r["admit"] - r["submit"] for r in res]) * 1e3
        span = max(r["done"] for r in res) - min(r["submit"] for r in res)
        return {"pairs_per_s": total_pairs / span, "wall_s": t1 - t0,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "admit_wait_p99_ms": float(np.percentile(wait, 99)),
                "batches": st["batches"] - st0["batches"],
                "engine_busy_s": st["busy_s"] - st0["busy_s"]}

    free_b, total_b = torch.cuda.mem_get_info()
    log(f"serving: {n_req} requests, {total_pairs} pairs; device memory free "
        f"{free_b / 2**30:.1f} of {total_b / 2**30:.1f} GiB; saturation run")
    sat = run(np.zeros(n_req), check=True)
    log(f"serving saturation: {sat}")
    sat_req_rate = n_req / (sat["wall_s"])
    unit_gaps = rng.exponential(1.0, n_req)  # one arrival pattern, scaled per load
    swept, loaded = [], None
    order = list(sweep) + ([] if load in sweep else [load])
    for f in order:
        lam = f * sat_req_rate
        free_b, _ = torch.cuda.mem_get_info()
        log(f"serving at load {f}: device memory free {free_b / 2**30:.1f} GiB")
        r = run(unit_gaps / lam)
        r.update({"offered_load": f, "offered_req_per_s": lam,
                  "offered_pairs_per_s": f * sat_req_rate * total_pairs / n_req})
        log(f"serving at load {f}: {r}")
        swept.append(r)
        if f == load and loaded is None:
            loaded = r
    max_reserved = srv.stats()["max_reserved_bytes"] / 2**30
    srv.close()
    return {"workload": "serving_mix: Poisson requests of 1-4096 pairs (log-uniform), "
                        "100-10,000 bp log-uniform, 1-10 % edits, CIGAR",
            "requests": n_req, "pairs": total_pairs, "budget_gib": 64, "streams": 4,
            "max_chunk_pairs": chunk, "options": "defaults (chosen per batch)",
            "max_reserved_gib": max_reserved,
            "saturation": sat, "offered_load": load, "offered_req_per_s": loaded["offered_req_per_s"],
            "at_load": loaded, "sweep": swept,
            "p50_ms": loaded["p50_ms"], "p99_ms": loaded["p99_ms"]}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(pairs shard across GPUs with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    import paper_2204_02085_amd as wfa

    if args.calib_copy_mib:
        # a plain copy of known size, for scaling the HBM byte counters
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: 3 x {args.calib_copy_mib} MiB device to device")
        del src, dst
    if args.calib_read_mib:
        # a reduction reads its input once and writes a few bytes
        x = torch.ones((args.calib_read_mib << 20) // 4, dtype=torch.int32, device="cuda")
        for _ in range(3):
            tot = int(x.sum().item())
        torch.cuda.synchronize()
        log(f"calibration read: 3 x {args.calib_read_mib} MiB summed ({tot} ones)")
        del x

    t_gen = time.perf_counter()
    batch = synth.workload(args.workload, args.pairs)
    t_gen = time.perf_counter() - t_gen
    n = len(batch)
    al = wfa.Aligner(0)
    if args.encoding == "packed2":
        enc = wfa.WFA_PACKED2
        pat, txt, pairs = al.to_device_packed(batch)
    else:
        enc = wfa.WFA_ASCII
        pat, txt, pairs = al.to_device(batch)
    torch.cuda.synchronize()
    # room for every run: ~40 per 100 bp pair, a quarter of the bases for long pairs
    cap = int(max(n * 40, int(((batch.p_len.astype(np.int64) + batch.t_len) // 4 + 8).sum()))) + 1024
    scores, runs, offsets = al.alloc_outputs(n, cap, True)
    dev = (pat, txt, pairs, scores, runs, offsets)

    # the autotuner picks the launch options on a sample of this batch
    # (outside the timed region); every candidate must give identical bytes
    log(f"generated {n} pairs in {t_gen:.1f} s; autotuning")
    t_tune = time.perf_counter()
    if args.options:
        tuned = {k: int(v) for k, v in json.loads(args.options).items()}
    else:
        tuned = tune_on_disjoint_sample(al, wfa, synth, args.workload, n, args.tune_sample or n, enc,
                                        args.mode == "cigar")
    t_tune = time.perf_counter() - t_tune

    log(f"autotuned in {t_tune:.1f} s: {tuned}; timing {args.steps} steps")
    cig = args.mode == "cigar"
    el, kms, st = time_schedule(al, dev, n, args.steps, args.warmup, tuned, enc, cig)
    log(f"tuned: {n * args.steps / el / 1e6:.1f} M pairs/s")
    ms_step = el / args.steps * 1e3
    value = n * args.steps / el
    needed = al.last_needed()
    tuned_stats = st
    got_scores = scores.cpu().numpy().copy()
    got_offsets = offsets.cpu().numpy().view(np.uint64).copy()

    # the dominant kernel alone: the same launch with the work before and
    # after it replayed as two graphs, so that events the library records
    # around the kernel on its stream time it alone
    kel, kms_k, kst = time_schedule(al, dev, n, args.steps, 1, {**tuned, "use_graph": 2}, enc, cig)
    kernel_ms = float(np.mean(kms_k))
    log(f"kernel alone: {kernel_ms:.3f} ms per launch (whole call {ms_step:.3f} ms)")

    # default knobs (the library's own per-batch choice, no tuning)
    default_value = None
    if args.plain_steps > 0:
        del_el, _, _ = time_schedule(al, dev, n, args.plain_steps, 1, {}, enc, cig)
        default_value = n * args.plain_steps / del_el
        log(f"default knobs: {default_value / 1e6:.1f} M pairs/s")

    # the same launch shape (window, lanes, step cap, workgroup size) as one
    # persistent bucketed launch replayed through graphs, and as the plain
    # per-batch kernel
    batched = None
    if args.plain_steps > 0:
        log("timing persistent and plain schedules")
        shape = {k: tuned.get(k, 0) for k in ("window", "lanes_per_pair", "step_cap",
                                              "block_threads")}
        shape["lane_kernel"] = tuned.get("lane_kernel", 0)
        bel, bkms, bst = time_schedule(al, dev, n, args.plain_steps, 1,
                                       {**shape, "schedule": wfa.WFA_SCHED_PERSISTENT,
                                        "bucket": 1, "use_graph": 1}, enc, cig)
        batched_value = n * args.plain_steps / bel
        pel, pkms, pst = time_schedule(al, dev, n, args.plain_steps, 1,
                                       {**shape, "schedule": wfa.WFA_SCHED_PLAIN,
                                        "bucket": -1, "use_graph": -1}, enc, cig)
        plain_value = n * args.plain_steps / pel
        if not np.array_equal(scores.cpu().numpy(), got_scores):
            raise RuntimeError("plain and tuned schedules disagree")
        batched = {"tuned_pairs_per_s": value,
                   "persistent_bucketed_graph_pairs_per_s": batched_value,
                   "plain_pairs_per_s": plain_value,
                   "speedup_persistent_vs_plain": batched_value / plain_value,
                   "speedup_tuned_vs_plain": value / plain_value,
                   "tuned_kernel_ms": kernel_ms,
                   "persistent_kernel_ms": float(np.mean(bkms)),
                   "plain_kernel_ms": float(np.mean(pkms)),
                   "launch_shape": shape}

    # results of both schedules are identical (cheap check on the last step)
    torch.cuda.synchronize()

    gcups = float((batch.p_len.astype(np.float64) * batch.t_len.astype(np.float64)).sum()) \
        * args.steps / el / 1e9

    # CPU oracle on a bounded sample (also yields the algorithmic work counts)
    cpu = None
    cells_pp = windows_pp = None
    if args.cpu_pairs > 0:
        import oracle

        log("CPU oracle baseline")
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        sample = synth.workload(args.workload, min(args.cpu_pairs, n))
        t0 = time.perf_counter()
        ref = oracle.align_batch(sample, (4, 6, 2), cigar=args.mode == "cigar", threads=threads)
        t1 = time.perf_counter()
        cpu = {"value": len(sample) / (t1 - t0), "unit": "pairs/s", "cores": threads,
               "kind": "oracle",
               "sample": f"first {len(sample)} pairs of the same workload, score + CIGAR, "
                         f"{threads} threads, {t1 - t0:.2f} s wall "
                         f"({(t1 - t0) * threads:.1f} thread-seconds)"}
        cells_pp = ref.stats["cells"] / len(sample)
        windows_pp = ref.stats["ext_windows"] / len(sample)
        # parity of the benchmarked batch: scores, CIGAR offsets and runs of
        # the sample's pairs, byte for byte; any difference ends the run
        k = len(sample)
        cig_ok = True
        if args.mode == "cigar":
            got_runs = runs[: int(got_offsets[k])].cpu().numpy().view(np.uint32)
            cig_ok = (np.array_equal(got_offsets[: k + 1], ref.offsets)
                      and np.array_equal(got_runs, ref.runs))
            del got_runs
        if not (np.array_equal(got_scores[:k], ref.scores) and cig_ok):
            print(f"bench: the timed batch differs from the oracle on its first {k} pairs",
                  file=sys.stderr)
            sys.exit(3)
        log(f"parity: the first {k} pairs of the timed batch equal the oracle byte for byte")

    host_path = None
    if args.host_steps > 0:
        log(f"host-memory path: {args.host_steps} calls")
        host_path, host_scores = host_path_run(al, wfa, batch, args.host_steps, tuned)
        if not np.array_equal(host_scores, got_scores):
            raise RuntimeError("host-memory path and device path disagree")

    # the second set of the configuration (5 M pairs of 100 bp at E = 2 %),
    # tuned and timed the same way; reported beside the headline
    second = None
    if args.second_set not in ("", "none") and args.second_set != args.workload:
        log(f"second set: {args.second_set}")
        del dev, pat, txt, pairs, scores, runs, offsets
        b2 = synth.workload(args.second_set, args.pairs)
        n2 = len(b2)
        if enc == wfa.WFA_PACKED2:
            p2, t2, d2 = al.to_device_packed(b2)
        else:
            p2, t2, d2 = al.to_device(b2)
        o2 = al.alloc_outputs(n2, n2 * 40 + 1024, True)
        tuned2 = tune_on_disjoint_sample(al, wfa, synth, args.second_set, n2,
                                         args.tune_sample or n2, enc)
        el2, kms2, st2 = time_schedule(al, (p2, t2, d2, *o2), n2, args.steps, args.warmup, tuned2,
                                       enc)
        second = {"workload": args.second_set, "pairs": n2, "pairs_per_s": n2 * args.steps / el2,
                  "ms_per_step": el2 / args.steps * 1e3, "kernel_ms": float(np.mean(kms2)),
                  "autotuned_options": tuned2}
        del p2, t2, d2, o2

    # the other configurations, for the record: 2 M uneven pairs (one
    # persistent bucketed graph-replayed launch, autotuned), 100 k long
    # pairs (general kernel), the main workload in score-only mode, the
    # main workload aligned ends-free (up to 10 bases of either sequence free
    # at either end, autotuned), and the WF-adaptive heuristic (minimum
    # wavefront length 10, distance threshold 50) on the long pairs and on
    # 1 M pairs of the main workload, each timed after one warm-up call; the
    # first pairs of each are checked against the oracle
    others = None
    if args.other_configs:
        import oracle

        others = {}
        for name, count, tune, modes, ends, heur in [
                ("uneven50_300_2m", 2_000_000, True, ("cigar",), None, None),
                ("long1k_10k_100k", 100_000, False, ("score", "cigar"), None, None),
                (args.workload, args.pairs, True, ("score",), None, None),
                (args.workload, args.pairs, True, ("cigar",), (10, 10, 10, 10), None),
                ("long1k_10k_100k", 100_000, False, ("score", "cigar"), None, (10, 50)),
                (args.workload, min(args.pairs, 1_000_000), False, ("cigar",), None, (10, 50))]:
            label = name if ends is None else name + "_ends_free_" + "_".join(map(str, ends))
            if name == args.workload and ends is None and heur is None:
                label = name + "_score_only"
            if heur is not None:
                label = name + "_adaptive_" + "_".join(map(str, heur))
            log(f"configuration {label}: {count} pairs")
            al.set_ends_free(*(ends or ()))
            al.set_heuristic(*(heur or ()))
            bo = synth.workload(name, count)
            no = len(bo)
            if enc == wfa.WFA_PACKED2:
                po, to, do_ = al.to_device_packed(bo)
            else:
                po, to, do_ = al.to_device(bo)
            rec = {"pairs": no}
            for mode in modes:
                cig = mode == "cigar"
                runs_cap = no * (40 if no > 1_000_000 else 1500) + 1024
                oo = al.alloc_outputs(no, runs_cap, cig)
                if tune:
                    al.set_ends_free(*(ends or ()))
                    opts = tune_on_disjoint_sample(al, wfa, synth, name, no,
                                                   min(args.tune_sample or no, no // 4), enc, cig)
                else:
                    opts = {}
                    al.set_options()
                al.set_options(**opts)
                steps = 3 if no > 1_000_000 else 1
                al.align_device(po, to, do_, no, *oo, (4, 6, 2), cig, enc)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    al.align_device(po, to, do_, no, *oo, (4, 6, 2), cig, enc)
                torch.cuda.synchronize()
                el = (time.perf_counter() - t0) / steps
                st = al.stats()
                rec[mode] = {"pairs_per_s": no / el, "ms_per_call": el * 1e3,
                             "short_pairs": st["short_pairs"], "general_pairs": st["general_pairs"],
                             "ms_short_kernel": st["ms_align"], "ms_general": st["ms_general"],
                             "options": opts or "defaults"}
                # the first pairs against the oracle (scores, and runs in CIGAR mode)
                k = min(no, 200 if "long" in name else 2000)
                sub = synth.workload(name, k)
                ref = oracle.align_batch(sub, (4, 6, 2), cigar=cig,
                                         threads=min(16, os.cpu_count() or 1), ends=ends,
                                         adaptive=heur, slot=int((sub.p_len.astype(np.int64)
                                                                  + sub.t_len).max()) + 1)
                ok = np.array_equal(oo[0][:k].cpu().numpy(), ref.scores)
                if cig and ok:
                    off = oo[2][: k + 1].cpu().numpy().view(np.uint64)
                    ok = (np.array_equal(off, ref.offsets) and np.array_equal(
                        oo[1][: int(off[k])].cpu().numpy().view(np.uint32), ref.runs))
                if not ok:
                    print(f"bench: configuration {label} ({mode}) differs from the oracle on its "
                          f"first {k} pairs", file=sys.stderr)
                    sys.exit(3)
                rec[mode]["oracle_checked_pairs"] = k
                del oo
            if ends is not None:
                rec["ends_free"] = list(ends)
            if heur is not None:
                rec["adaptive"] = {"min_wavefront_length": heur[0],
                                   "max_distance_threshold": heur[1]}
            others[label] = rec
            del po, to, do_, bo
        al.set_ends_free()
        al.set_heuristic()

    serving = None
    if args.serving_requests > 0:
        log(f"serving run: {args.serving_requests} requests")
        # server engines start from the context's options: the library's own
        # per-batch choice here, not a launch shape tuned for another workload
        al.set_options()
        al.set_ends_free()
        al.set_heuristic()
        sweep = () if args.serving_sweep == "none" else \
            tuple(float(v) for v in args.serving_sweep.split(",") if v.strip())
        serving = serving_run(al, wfa, synth, args.serving_requests, args.serving_load, sweep,
                              args.serving_chunk)

    roofline = None
    if cells_pp is not None and kernel_ms > 0:
        ops = n * (cells_pp * OPS_PER_CELL + windows_pp * OPS_PER_WINDOW)
        ops_itemised = n * (cells_pp * OPS_PER_CELL_ITEMISED + windows_pp * OPS_PER_WINDOW_ITEMISED)
        achieved = ops / (kernel_ms * 1e-3)
        prof = read_profile(kernel_source_hash(), kernel_label(kst))
        roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_INT_OPS / 1e12,
                    "unit": "Tops/s (int32 lane-ops)", "frac": achieved / PEAK_INT_OPS,
                    "traffic": prof.get("hbm_bytes_per_launch"),
                    "traffic_over_algorithmic": prof.get("traffic_over_algorithmic"),
                    "valu_issue_frac": prof.get("valu_issue_per_cu_cycle"),
                    "valu_insts_per_pair": prof.get("valu_insts_per_pair"),
                    "kernel": kernel_label(kst),
                    "kernel_ms": kernel_ms, "ops_per_launch": ops,
                    "cost_model": f"{OPS_PER_CELL} ops per cell + {OPS_PER_WINDOW} per 32-base "
                                  "extension compare",
                    "frac_itemised_model": ops_itemised / (kernel_ms * 1e-3) / PEAK_INT_OPS,
                    "cells_per_pair": cells_pp, "windows_per_pair": windows_pp}

    out = {
        "metric": "aligned pairs/s (100bp E=4%, CIGAR), batched vs plain; p99 latency",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "pairs": n, "read_length": 100,
                   "edits": 4 if "e4" in args.workload else 2, "penalties": [4, 6, 2],
                   "mode": args.mode,
                   "input": ("2-bit packed uint64 words in HBM" if enc == wfa.WFA_PACKED2
                             else "ASCII in HBM"),
                   "schedule": "autotuned (see autotuned_options)"},
        "gcups_equivalent": gcups,
        "cigar_runs": needed,
        "autotuned_options": tuned,
        "autotune_seconds": t_tune,
        "autotune_sample": f"{args.tune_sample or n} pairs of the same stream after the timed batch",
        "default_knobs_pairs_per_s": default_value,
        "batched_vs_plain": batched,
        "phase_ms": {k: tuned_stats[k] for k in ("ms_pack", "ms_align", "ms_general", "ms_compact",
                                                 "ms_total")},
        "second_set": second,
        "other_configs": others,
        "host_path": host_path,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
        "gen_seconds": t_gen,
    }
    al.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
