"""Python binding of libwfa (batched gap-affine WFA on MI355X / gfx950).

Argument marshalling only: every step of the alignment runs in the HIP
kernels behind the C ABI declared in ``include/wfa.h``.  The functions below
carry the C names; ``Aligner`` adds a convenience layer that moves numpy
arrays into torch device tensors (PyTorch provides device memory and
streams, nothing else).

The library must be built (``python paper_2204_02085_amd/build.py``); if it
is missing, importing the binding raises ``ImportError`` -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwfa.so")

# ---- C types (mirror include/wfa.h) -----------------------------------------
WFA_SCORE, WFA_CIGAR = 0, 1
WFA_ASCII, WFA_PACKED2 = 0, 1
WFA_HOST, WFA_DEVICE = 0, 1
WFA_SCHED_AUTO, WFA_SCHED_PLAIN, WFA_SCHED_PERSISTENT, WFA_SCHED_GENERAL = 0, 1, 2, 3
WFA_OK, WFA_E_INVAL, WFA_E_ALPHABET, WFA_E_NOMEM = 0, -1, -2, -3
WFA_E_CAPACITY, WFA_E_DEVICE, WFA_E_TOO_LONG, WFA_E_BUSY, WFA_E_NOTFOUND = -4, -5, -6, -7, -8
WFA_E_LIMIT = -9
WFA_OP_MATCH, WFA_OP_MISMATCH, WFA_OP_INS, WFA_OP_DEL = 0, 1, 2, 3
WFA_MAX_LENGTH = 1 << 26

EXPORTED = [
    "wfa_ctx_create", "wfa_ctx_destroy", "wfa_set_options", "wfa_set_ends_free",
    "wfa_set_heuristic", "wfa_align_batch",
    "wfa_copy_last_cigars", "wfa_host_alloc", "wfa_host_free", "wfa_pack2bit", "wfa_autotune",
    "wfa_last_stats", "wfa_strerror",
    "wfa_server_open", "wfa_server_submit", "wfa_server_poll", "wfa_server_release",
    "wfa_server_estimate_bytes", "wfa_server_get_stats", "wfa_server_close",
    "wfa_align_batch_noalloc",
]
WFA_NOALLOC_SCRATCH_BYTES = 128 << 20
WFA_NOALLOC_MAX_PAIRS = 1 << 18

PAIR_DTYPE = np.dtype([("p_start", "<u8"), ("t_start", "<u8"), ("p_len", "<u4"),
                       ("t_len", "<u4")])


class wfa_penalties(ctypes.Structure):
    _fields_ = [("mismatch", ctypes.c_int32), ("gap_open", ctypes.c_int32),
                ("gap_extend", ctypes.c_int32)]


class wfa_options(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("window", ctypes.c_int32),
                ("step_cap", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("bucket", ctypes.c_int32), ("general_pairs", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("lanes_per_pair", ctypes.c_int32),
                ("host_chunk_pairs", ctypes.c_int32), ("cascade_window", ctypes.c_int32),
                ("general_slice_kib", ctypes.c_int32), ("lane_kernel", ctypes.c_int32),
                ("general_step_limit", ctypes.c_int32), ("general_checkpoint", ctypes.c_int32)]


class wfa_ends_free(ctypes.Structure):
    _fields_ = [("pattern_begin_free", ctypes.c_uint32), ("pattern_end_free", ctypes.c_uint32),
                ("text_begin_free", ctypes.c_uint32), ("text_end_free", ctypes.c_uint32)]


class wfa_heuristic(ctypes.Structure):
    _fields_ = [("min_wavefront_length", ctypes.c_int32), ("max_distance_threshold", ctypes.c_int32)]


class wfa_stats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_uint64), ("short_pairs", ctypes.c_uint64),
                ("general_pairs", ctypes.c_uint64), ("requeued", ctypes.c_uint64),
                ("cigar_runs", ctypes.c_uint64), ("window", ctypes.c_int32),
                ("lanes_per_pair", ctypes.c_int32), ("host_chunks", ctypes.c_int32),
                ("step_cap", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("graph_replayed", ctypes.c_int32), ("ms_pack", ctypes.c_double),
                ("ms_align", ctypes.c_double), ("ms_general", ctypes.c_double),
                ("ms_compact", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("cascade_window", ctypes.c_int32), ("lane_kernel", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class wfa_request(ctypes.Structure):
    _fields_ = [("patterns", ctypes.c_void_p), ("texts", ctypes.c_void_p),
                ("pairs", ctypes.c_void_p), ("num_pairs", ctypes.c_size_t)]


wfa_executor_fn = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(wfa_request),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint32),
                                   ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint64),
                                   ctypes.POINTER(ctypes.c_size_t))


class wfa_server_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("streams", ctypes.c_int32),
                ("max_chunk_pairs", ctypes.c_int32), ("queue_limit", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("pen", wfa_penalties),
                ("executor", wfa_executor_fn), ("executor_user", ctypes.c_void_p)]


class wfa_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("pairs", ctypes.c_uint64),
                ("budget_bytes", ctypes.c_size_t), ("reserved_bytes", ctypes.c_size_t),
                ("max_reserved_bytes", ctypes.c_size_t), ("busy_s", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class wfa_result(ctypes.Structure):
    _fields_ = [("num_pairs", ctypes.c_size_t), ("scores", ctypes.POINTER(ctypes.c_int32)),
                ("cigar_runs", ctypes.POINTER(ctypes.c_uint32)),
                ("cigar_offsets", ctypes.POINTER(ctypes.c_uint64)),
                ("submit_time_s", ctypes.c_double), ("admit_time_s", ctypes.c_double),
                ("done_time_s", ctypes.c_double), ("status", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python paper_2204_02085_amd/build.py`")
    # torch ships its own HIP runtime under the same soname; load it first so
    # that the process holds exactly one HIP runtime, shared with torch.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    p, i32, i64, u64, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                            ctypes.c_size_t)
    sig = {
        "wfa_ctx_create": ([ctypes.c_int, sz, ctypes.POINTER(p)], ctypes.c_int),
        "wfa_ctx_destroy": ([p], None),
        "wfa_set_options": ([p, ctypes.POINTER(wfa_options)], ctypes.c_int),
        "wfa_set_ends_free": ([p, ctypes.POINTER(wfa_ends_free)], ctypes.c_int),
        "wfa_set_heuristic": ([p, ctypes.POINTER(wfa_heuristic)], ctypes.c_int),
        "wfa_align_batch": ([p, p, p, p, sz, ctypes.c_int, ctypes.c_int, wfa_penalties,
                             ctypes.c_int, p, p, sz, p, ctypes.POINTER(sz),
                             ctypes.POINTER(i64), p], ctypes.c_int),
        "wfa_copy_last_cigars": ([p, p, sz, p], ctypes.c_int),
        "wfa_align_batch_noalloc": ([p, p, p, p, sz, ctypes.c_int, wfa_penalties, ctypes.c_int,
                                     p, p, sz, p, ctypes.POINTER(sz), ctypes.POINTER(i64), p],
                                    ctypes.c_int),
        "wfa_host_alloc": ([sz, ctypes.POINTER(p)], ctypes.c_int),
        "wfa_host_free": ([p], None),
        "wfa_pack2bit": ([p, p, p, p, sz, p, sz, p, ctypes.POINTER(sz), ctypes.POINTER(i64), p],
                         ctypes.c_int),
        "wfa_autotune": ([p, p, p, p, sz, ctypes.c_int, ctypes.c_int, wfa_penalties, ctypes.c_int,
                          sz, ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(wfa_options)],
                         ctypes.c_int),
        "wfa_last_stats": ([p, ctypes.POINTER(wfa_stats)], ctypes.c_int),
        "wfa_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "wfa_server_open": ([p, ctypes.POINTER(wfa_server_cfg), ctypes.POINTER(p)], ctypes.c_int),
        "wfa_server_submit": ([p, ctypes.POINTER(wfa_request), ctypes.POINTER(u64)],
                              ctypes.c_int),
        "wfa_server_poll": ([p, u64, i64, ctypes.POINTER(wfa_result)], ctypes.c_int),
        "wfa_server_release": ([p, u64], ctypes.c_int),
        "wfa_server_estimate_bytes": ([p, ctypes.POINTER(wfa_request)], sz),
        "wfa_server_get_stats": ([p, ctypes.POINTER(wfa_server_stats)], ctypes.c_int),
        "wfa_server_close": ([p], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    del i32, u64
    return lib


lib = _load()

# C entry points under their own names
wfa_ctx_create = lib.wfa_ctx_create
wfa_ctx_destroy = lib.wfa_ctx_destroy
wfa_set_options = lib.wfa_set_options
wfa_set_ends_free = lib.wfa_set_ends_free
wfa_set_heuristic = lib.wfa_set_heuristic
wfa_align_batch = lib.wfa_align_batch
wfa_copy_last_cigars = lib.wfa_copy_last_cigars
wfa_align_batch_noalloc = lib.wfa_align_batch_noalloc
wfa_host_alloc = lib.wfa_host_alloc
wfa_host_free = lib.wfa_host_free
wfa_pack2bit = lib.wfa_pack2bit
wfa_autotune = lib.wfa_autotune
wfa_last_stats = lib.wfa_last_stats
wfa_strerror = lib.wfa_strerror
wfa_server_open = lib.wfa_server_open
wfa_server_submit = lib.wfa_server_submit
wfa_server_poll = lib.wfa_server_poll
wfa_server_release = lib.wfa_server_release
wfa_server_estimate_bytes = lib.wfa_server_estimate_bytes
wfa_server_get_stats = lib.wfa_server_get_stats
wfa_server_close = lib.wfa_server_close


class WFAError(RuntimeError):
    def __init__(self, status: int, what: str = "", bad: int = -1):
        msg = wfa_strerror(status).decode()
        super().__init__(f"{what}: {msg} (status {status}{', pair ' + str(bad) if bad >= 0 else ''})")
        self.status = status
        self.bad = bad


def host_empty(shape, dtype) -> np.ndarray:
    """Uninitialised numpy array in page-locked host memory (wfa_host_alloc),
    released with wfa_host_free once the array and all its views are gone.
    Host-memory batches whose buffers come from here copy at the full link
    rate."""
    dt = np.dtype(dtype)
    shape = (int(shape),) if np.isscalar(shape) else tuple(int(x) for x in shape)
    nbytes = int(np.prod(shape, dtype=np.int64)) * dt.itemsize
    ptr = ctypes.c_void_p()
    rc = wfa_host_alloc(nbytes, ctypes.byref(ptr))
    if rc != WFA_OK:
        raise WFAError(rc, "wfa_host_alloc")
    buf = (ctypes.c_uint8 * max(nbytes, 1)).from_address(ptr.value)
    weakref.finalize(buf, wfa_host_free, ptr.value)
    return np.frombuffer(buf, dtype=np.uint8, count=nbytes).view(dt).reshape(shape)


def host_copy(a) -> np.ndarray:
    """`a` copied into page-locked host memory (see host_empty)."""
    a = np.ascontiguousarray(a)
    out = host_empty(a.shape, a.dtype)
    out[...] = a
    return out


def pairs_array(p_off, p_len, t_off, t_len) -> np.ndarray:
    """Descriptor array (wfa_pair layout) from per-pair starts and lengths."""
    a = np.zeros(len(p_len), dtype=PAIR_DTYPE)
    a["p_start"] = p_off
    a["t_start"] = t_off
    a["p_len"] = p_len
    a["t_len"] = t_len
    return a


class Aligner:
    """One library context on one GPU, with device-resident batches.

    ``align`` takes a batch with numpy fields (``patterns``, ``texts``,
    ``p_off``, ``p_len``, ``t_off``, ``t_len``; e.g. ``synth.Batch``), copies
    it to the device with torch, and returns numpy (scores, runs, offsets).
    ``align_device`` works on torch device tensors already in HBM.
    """

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        import torch

        self.torch = torch
        self.device = device
        torch.cuda.set_device(device)
        ctx = ctypes.c_void_p()
        rc = wfa_ctx_create(device, hbm_budget_bytes, ctypes.byref(ctx))
        if rc != WFA_OK:
            raise WFAError(rc, "wfa_ctx_create")
        self.ctx = ctx
        self._servers = weakref.WeakSet()  # servers open on this context

    def close(self):
        if getattr(self, "ctx", None):
            # a closing server hands its engines to the context, so every
            # server goes before the context does
            for srv in list(getattr(self, "_servers", ())):
                srv.close()
            wfa_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_options(self, **kw):
        o = wfa_options(**kw)
        rc = wfa_set_options(self.ctx, ctypes.byref(o))
        if rc != WFA_OK:
            raise WFAError(rc, "wfa_set_options")

    def set_ends_free(self, pattern_begin=0, pattern_end=0, text_begin=0, text_end=0):
        """Ends-free alignment for later calls (all zero: global)."""
        ef = wfa_ends_free(pattern_begin, pattern_end, text_begin, text_end)
        rc = wfa_set_ends_free(self.ctx, ctypes.byref(ef))
        if rc != WFA_OK:
            raise WFAError(rc, "wfa_set_ends_free")

    def set_heuristic(self, min_wavefront_length=0, max_distance_threshold=0):
        """WF-adaptive heuristic for later calls (min_wavefront_length 0: exact)."""
        h = wfa_heuristic(min_wavefront_length, max_distance_threshold)
        rc = wfa_set_heuristic(self.ctx, ctypes.byref(h))
        if rc != WFA_OK:
            raise WFAError(rc, "wfa_set_heuristic")

    def autotune(self, patterns, texts, pairs, n, penalties=(4, 6, 2), cigar=True,
                 encoding=WFA_ASCII, sample_pairs=0, cache_path=None, force=False) -> dict:
        """wfa_autotune on device tensors; returns the chosen options."""
        o = wfa_options()
        rc = wfa_autotune(self.ctx, patterns.data_ptr(), texts.data_ptr(), pairs.data_ptr(), n,
                          encoding, WFA_DEVICE, wfa_penalties(*penalties),
                          WFA_CIGAR if cigar else WFA_SCORE, sample_pairs,
                          cache_path.encode() if cache_path else None, int(force), ctypes.byref(o))
        if rc != WFA_OK:
            raise WFAError(rc, "wfa_autotune")
        return {f: getattr(o, f) for f, _ in o._fields_}

    def stats(self) -> dict:
        s = wfa_stats()
        wfa_last_stats(self.ctx, ctypes.byref(s))
        return s.as_dict()

    def to_device(self, batch):
        """Device tensors (patterns, texts, pairs) for a numpy batch."""
        t = self.torch
        dev = f"cuda:{self.device}"
        pairs = pairs_array(batch.p_off, batch.p_len, batch.t_off, batch.t_len)
        return (t.from_numpy(np.ascontiguousarray(batch.patterns)).to(dev),
                t.from_numpy(np.ascontiguousarray(batch.texts)).to(dev),
                t.from_numpy(pairs.view(np.uint8).copy()).to(dev))

    def pack2bit(self, ascii, starts, lens):
        """wfa_pack2bit on device tensors (uint8 ASCII, int64 starts, int32
        lengths); returns (int64 words, int64 word starts) on the device."""
        t = self.torch
        n = int(lens.numel())
        nwords = int(((lens.to(t.int64) + 31) // 32).sum().item()) + 8
        words = t.empty(nwords, dtype=t.int64, device=ascii.device)
        ws = t.empty(n + 1, dtype=t.int64, device=ascii.device)
        total = ctypes.c_size_t(0)
        bad = ctypes.c_int64(-1)
        rc = wfa_pack2bit(self.ctx, ascii.data_ptr(), starts.data_ptr(), lens.data_ptr(), n,
                          words.data_ptr(), nwords, ws.data_ptr(), ctypes.byref(total),
                          ctypes.byref(bad), t.cuda.current_stream(self.device).cuda_stream)
        if rc != WFA_OK:
            raise WFAError(rc, "wfa_pack2bit", bad.value)
        return words, ws

    def to_device_packed(self, batch):
        """Device tensors (pattern words, text words, pairs) with both sides
        packed to 2-bit words by the library; pair starts are word indices."""
        t = self.torch
        dev = f"cuda:{self.device}"
        out = []
        for seqs, off, ln in ((batch.patterns, batch.p_off, batch.p_len),
                              (batch.texts, batch.t_off, batch.t_len)):
            ascii = t.from_numpy(np.ascontiguousarray(seqs)).to(dev)
            starts = t.from_numpy(np.ascontiguousarray(off).view(np.int64)).to(dev)
            lens = t.from_numpy(np.ascontiguousarray(ln).view(np.int32)).to(dev)
            words, ws = self.pack2bit(ascii, starts, lens)
            del ascii
            out.append((words, ws[: len(ln)].cpu().numpy().view(np.uint64)))
        pairs = pairs_array(out[0][1], batch.p_len, out[1][1], batch.t_len)
        return out[0][0], out[1][0], t.from_numpy(pairs.view(np.uint8).copy()).to(dev)

    def alloc_outputs(self, n: int, capacity: int, cigar: bool = True):
        t = self.torch
        dev = f"cuda:{self.device}"
        scores = t.empty(n, dtype=t.int32, device=dev)
        offsets = t.empty(n + 1, dtype=t.int64, device=dev) if cigar else None
        runs = t.empty(max(capacity, 1), dtype=t.int32, device=dev) if cigar else None
        return scores, runs, offsets

    def align_device(self, patterns, texts, pairs, n, scores, runs=None, offsets=None,
                     penalties=(4, 6, 2), cigar=True, encoding=WFA_ASCII, stream=None):
        """Run wfa_align_batch on device tensors; returns runs needed."""
        t = self.torch
        needed = ctypes.c_size_t(0)
        bad = ctypes.c_int64(-1)
        if stream is None:
            stream = t.cuda.current_stream(self.device).cuda_stream
        rc = wfa_align_batch(
            self.ctx, patterns.data_ptr(), texts.data_ptr(), pairs.data_ptr(), n, encoding,
            WFA_DEVICE, wfa_penalties(*penalties), WFA_CIGAR if cigar else WFA_SCORE,
            scores.data_ptr(), runs.data_ptr() if cigar else None,
            runs.numel() if cigar else 0, offsets.data_ptr() if cigar else None,
            ctypes.byref(needed), ctypes.byref(bad), stream)
        self._needed = needed.value
        if rc != WFA_OK:
            raise WFAError(rc, "wfa_align_batch", bad.value)
        return needed.value

    def align(self, batch, penalties=(4, 6, 2), cigar=True, capacity=None):
        """Align a numpy batch on the GPU; returns numpy scores, runs, offsets."""
        n = len(batch.p_len)
        pat, txt, pairs = self.to_device(batch)
        if capacity is None:
            capacity = int(n * 24 + 1024)
        scores, runs, offsets = self.alloc_outputs(n, capacity, cigar)
        try:
            needed = self.align_device(pat, txt, pairs, n, scores, runs, offsets, penalties, cigar)
        except WFAError as e:
            if e.status != WFA_E_CAPACITY:
                raise
            runs = self.torch.empty(int(self.last_needed()), dtype=self.torch.int32,
                                    device=scores.device)
            rc = wfa_copy_last_cigars(self.ctx, runs.data_ptr(), runs.numel(),
                                      offsets.data_ptr())
            if rc != WFA_OK:
                raise WFAError(rc, "wfa_copy_last_cigars")
            needed = runs.numel()
        self.torch.cuda.synchronize(self.device)
        sc = scores.cpu().numpy()
        if not cigar:
            return sc, None, None
        off = offsets.cpu().numpy().astype(np.uint64)
        rr = runs[:needed].cpu().numpy().view(np.uint32).copy()
        return sc, rr, off

    def last_needed(self) -> int:
        return int(getattr(self, "_needed", 0))

    def align_host(self, batch, penalties=(4, 6, 2), cigar=True, encoding=WFA_ASCII,
                   capacity=None, pinned=False, patterns=None, texts=None):
        """Host-memory variant (the library's chunk pipeline moves the data).
        `patterns` / `texts` replace the batch's own buffers (e.g. 2-bit
        words for WFA_PACKED2, with p_off / t_off in words); pinned=True puts
        the outputs in page-locked memory.  If the runs exceed `capacity` they
        are fetched with wfa_copy_last_cigars."""
        n = len(batch.p_len)
        pairs = pairs_array(batch.p_off, batch.p_len, batch.t_off, batch.t_len)
        pat = batch.patterns if patterns is None else patterns
        txt = batch.texts if texts is None else texts
        empty = host_empty if pinned else np.empty
        scores = empty(n, np.int32)
        offsets = empty(n + 1, np.uint64)
        cap = n * 24 + 1024 if capacity is None else int(capacity)
        runs = empty(max(cap, 1), np.uint32)
        needed = ctypes.c_size_t(0)
        bad = ctypes.c_int64(-1)
        rc = wfa_align_batch(
            self.ctx, pat.ctypes.data, txt.ctypes.data, pairs.ctypes.data, n,
            encoding, WFA_HOST, wfa_penalties(*penalties), WFA_CIGAR if cigar else WFA_SCORE,
            scores.ctypes.data, runs.ctypes.data if cigar else None, cap if cigar else 0,
            offsets.ctypes.data if cigar else None, ctypes.byref(needed), ctypes.byref(bad), None)
        self._needed = needed.value
        if cigar and rc == WFA_E_CAPACITY:
            runs = empty(max(needed.value, 1), np.uint32)
            rc = wfa_copy_last_cigars(self.ctx, runs.ctypes.data, needed.value, None)
            if rc != WFA_OK:
                raise WFAError(rc, "wfa_copy_last_cigars")
        elif rc != WFA_OK:
            raise WFAError(rc, "wfa_align_batch", bad.value)
        if not cigar:
            return scores, None, None
        return scores, runs[:needed.value].copy(), offsets


class Server:
    """Continuous-batching alignment server (wraps wfa_server_*).

    ``aligner`` supplies the GPU context; with ``executor`` (a Python callable
    ``f(batch_dict) -> (scores, runs, offsets)``) the scheduler runs without a
    GPU, which is how its admission and batching logic is tested on a CPU.
    """

    def __init__(self, aligner=None, hbm_budget_bytes=0, streams=4, max_chunk_pairs=65536,
                 penalties=(4, 6, 2), cigar=True, executor=None, queue_limit=0):
        cfg = wfa_server_cfg()
        cfg.hbm_budget_bytes = hbm_budget_bytes
        cfg.streams = streams
        cfg.max_chunk_pairs = max_chunk_pairs
        cfg.queue_limit = queue_limit
        cfg.mode = WFA_CIGAR if cigar else WFA_SCORE
        cfg.pen = wfa_penalties(*penalties)
        self.cigar = cigar
        self._keep = []
        if executor is not None:
            def trampoline(user, req, scores, runs, cap, offsets, needed):
                try:
                    r = req.contents
                    n = r.num_pairs
                    pairs = np.ctypeslib.as_array(
                        ctypes.cast(r.pairs, ctypes.POINTER(ctypes.c_uint8)),
                        shape=(n * PAIR_DTYPE.itemsize,)).view(PAIR_DTYPE)
                    plen_total = int((pairs["p_start"] + pairs["p_len"]).max(initial=0))
                    tlen_total = int((pairs["t_start"] + pairs["t_len"]).max(initial=0))
                    pat = np.ctypeslib.as_array(ctypes.cast(r.patterns, ctypes.POINTER(ctypes.c_uint8)),
                                                shape=(max(plen_total, 1),))
                    txt = np.ctypeslib.as_array(ctypes.cast(r.texts, ctypes.POINTER(ctypes.c_uint8)),
                                                shape=(max(tlen_total, 1),))
                    sc, rr, off = executor(dict(patterns=pat, texts=txt, pairs=pairs.copy()))
                    for i in range(n):
                        scores[i] = int(sc[i])
                    if self.cigar:
                        needed[0] = len(rr)
                        if len(rr) > cap:
                            return WFA_E_CAPACITY
                        for i in range(len(rr)):
                            runs[i] = int(rr[i])
                        for i in range(n + 1):
                            offsets[i] = int(off[i])
                    return WFA_OK
                except Exception:  # noqa: BLE001 - reported as a device error
                    import traceback

                    traceback.print_exc()
                    return WFA_E_DEVICE

            fn = wfa_executor_fn(trampoline)
            self._keep.append(fn)
            cfg.executor = fn
        ctx = aligner.ctx if aligner is not None else None
        srv = ctypes.c_void_p()
        rc = wfa_server_open(ctx, ctypes.byref(cfg), ctypes.byref(srv))
        if rc != WFA_OK:
            raise WFAError(rc, "wfa_server_open")
        self.srv = srv
        # the context must outlive the server: keep it, and let it close us first
        self._aligner = aligner
        if aligner is not None:
            aligner._servers.add(self)

    def _request(self, batch):
        pairs = pairs_array(batch.p_off, batch.p_len, batch.t_off, batch.t_len)
        pat = np.ascontiguousarray(batch.patterns)
        txt = np.ascontiguousarray(batch.texts)
        req = wfa_request(pat.ctypes.data, txt.ctypes.data, pairs.ctypes.data, len(pairs))
        return req, (pat, txt, pairs)

    def submit(self, batch) -> int:
        req, keep = self._request(batch)
        t = ctypes.c_uint64(0)
        rc = wfa_server_submit(self.srv, ctypes.byref(req), ctypes.byref(t))
        if rc != WFA_OK:
            raise WFAError(rc, "wfa_server_submit")
        del keep  # the server copied the request
        return t.value

    def estimate_bytes(self, batch) -> int:
        req, keep = self._request(batch)
        return int(wfa_server_estimate_bytes(self.srv, ctypes.byref(req)))

    def poll(self, ticket: int, timeout_us: int = -1):
        """Result dict of a finished ticket, or None on time-out."""
        res = wfa_result()
        rc = wfa_server_poll(self.srv, ticket, timeout_us, ctypes.byref(res))
        if rc == WFA_E_BUSY:
            return None
        if rc != WFA_OK:
            raise WFAError(rc, "wfa_server_poll")
        n = res.num_pairs
        out = {"status": res.status, "submit": res.submit_time_s, "admit": res.admit_time_s,
               "done": res.done_time_s, "num_pairs": n}
        out["scores"] = np.ctypeslib.as_array(res.scores, shape=(n,)).copy() if n else \
            np.zeros(0, np.int32)
        if self.cigar:
            off = np.ctypeslib.as_array(res.cigar_offsets, shape=(n + 1,)).copy()
            total = int(off[-1])
            out["offsets"] = off
            out["runs"] = np.ctypeslib.as_array(res.cigar_runs, shape=(total,)).copy() if total \
                else np.zeros(0, np.uint32)
        return out

    def release(self, ticket: int):
        wfa_server_release(self.srv, ticket)

    def stats(self) -> dict:
        st = wfa_server_stats()
        wfa_server_get_stats(self.srv, ctypes.byref(st))
        return st.as_dict()

    def close(self):
        if getattr(self, "srv", None):
            wfa_server_close(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
