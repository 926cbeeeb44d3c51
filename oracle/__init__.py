"""CPU oracle for batched gap-affine WFA alignment.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the benchmark's CPU-baseline leg, never by the library.  The arithmetic is
plain C in ``wfa_oracle.c`` (built with gcc, shares nothing with the HIP
library); this module only marshals arrays.

Pins (tests that tie the oracle to something other than itself) live in
``tests/test_oracle_pins.py``: brute-force enumeration of all alignments,
a textbook Gotoh dynamic program, the Levenshtein special case, closed
forms, CIGAR invariants and symmetry.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OP_M, OP_X, OP_I, OP_D = 0, 1, 2, 3
OP_CHARS = "MXID"


class Stats(ctypes.Structure):
    _fields_ = [
        ("cells", ctypes.c_int64),
        ("steps", ctypes.c_int64),
        ("ext_calls", ctypes.c_int64),
        ("ext_windows", ctypes.c_int64),
        ("ext_matches", ctypes.c_int64),
    ]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc."""
    src = os.path.join(_HERE, "wfa_oracle.c")
    hdr = os.path.join(_HERE, "wfa_oracle.h")
    newest = max(os.path.getmtime(src), os.path.getmtime(hdr))
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < newest:
        subprocess.check_call(["gcc", "-O2", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread",
                               "-o", _LIB_PATH, src])
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        p = ctypes.c_void_p
        i = ctypes.c_int
        i64 = ctypes.c_int64
        lib.oracle_align.argtypes = [p, i, p, i, i, i, i, i, p, p, i64, p, p]
        lib.oracle_align.restype = i
        lib.oracle_align_ends.argtypes = [p, i, p, i, i, i, i, i, i, i, i, i, p, p, i64, p, p]
        lib.oracle_align_ends.restype = i
        lib.oracle_align_batch.argtypes = [p, p, p, p, p, p, i64, i, i, i, i, p, p, i64, p, p,
                                           i, p]
        lib.oracle_align_batch.restype = i
        lib.oracle_align_batch_ends.argtypes = [p, p, p, p, p, p, i64, i, i, i, i, i, i, i, i, p,
                                                p, i64, p, p, i, p]
        lib.oracle_align_batch_ends.restype = i
        lib.oracle_align_adaptive.argtypes = [p, i, p, i, i, i, i, i, i, i, p, p, i64, p, p]
        lib.oracle_align_adaptive.restype = i
        lib.oracle_align_batch_adaptive.argtypes = [p, p, p, p, p, p, i64, i, i, i, i, i, i, p,
                                                    p, i64, p, p, i, p]
        lib.oracle_align_batch_adaptive.restype = i
        lib.oracle_pack2bit.argtypes = [p, i64, p, i64]
        lib.oracle_pack2bit.restype = i64
        _lib = lib
    return _lib


def _buf(b: bytes):
    return ctypes.create_string_buffer(b, len(b) + 1)


def align(pattern: bytes, text: bytes, penalties=(4, 6, 2), cigar: bool = True,
          with_stats: bool = False, ends=None, adaptive=None):
    """Align one pair.  Returns (score, runs) or (score, runs, stats).

    runs is a list of ``len << 4 | op`` words (empty in score-only mode).
    ends = (pattern_begin_free, pattern_end_free, text_begin_free,
    text_end_free) selects ends-free alignment (None: global).
    adaptive = (min_wavefront_length, max_distance_threshold) selects the
    WF-adaptive heuristic (global alignment only; None: exact).
    """
    lib = _load()
    x, o, e = penalties
    pb, pe, tb, te = (0, 0, 0, 0) if ends is None else ends
    n, m = len(pattern), len(text)
    cap = n + m + 1
    runs = (ctypes.c_uint32 * cap)()
    score = ctypes.c_int32(0)
    nr = ctypes.c_int64(0)
    st = Stats()
    if adaptive is not None:
        if ends is not None:
            raise ValueError("the adaptive heuristic applies to global alignment only")
        mwl, mdt = adaptive
        rc = lib.oracle_align_adaptive(_buf(pattern), n, _buf(text), m, x, o, e, mwl, mdt,
                                       int(cigar), ctypes.byref(score), runs, cap,
                                       ctypes.byref(nr), ctypes.byref(st))
    else:
        rc = lib.oracle_align_ends(_buf(pattern), n, _buf(text), m, x, o, e, pb, pe, tb, te,
                                   int(cigar), ctypes.byref(score), runs, cap, ctypes.byref(nr),
                                   ctypes.byref(st))
    if rc != 0:
        raise ValueError(f"oracle_align failed with status {rc}")
    out = [int(runs[j]) for j in range(nr.value)]
    if with_stats:
        return score.value, out, st.as_dict()
    return score.value, out


@dataclass
class BatchResult:
    scores: np.ndarray  # int32 [N]
    runs: np.ndarray  # uint32, compacted
    offsets: np.ndarray  # uint64 [N+1]
    stats: dict


def align_batch(batch, penalties=(4, 6, 2), cigar: bool = True, threads: int = 1,
                slot: int | None = None, ends=None, adaptive=None) -> BatchResult:
    """Align every pair of a ``synth.Batch`` on `threads` host threads
    (`ends` and `adaptive` as in ``align``)."""
    lib = _load()
    x, o, e = penalties
    pb, pe, tb, te = (0, 0, 0, 0) if ends is None else ends
    N = len(batch)
    if slot is None:
        slot = int((batch.p_len.astype(np.int64) + batch.t_len.astype(np.int64)).max(initial=0)) + 1
        slot = min(slot, 4096)
    scores = np.zeros(N, dtype=np.int32)
    nruns = np.zeros(N, dtype=np.int64)
    status = np.zeros(N, dtype=np.int32)
    runs = np.zeros(N * slot if cigar else 1, dtype=np.uint32)
    st = Stats()
    if adaptive is not None:
        if ends is not None:
            raise ValueError("the adaptive heuristic applies to global alignment only")
        mwl, mdt = adaptive
        rc = lib.oracle_align_batch_adaptive(
            batch.patterns.ctypes.data, batch.p_off.ctypes.data, batch.p_len.ctypes.data,
            batch.texts.ctypes.data, batch.t_off.ctypes.data, batch.t_len.ctypes.data, N, x, o,
            e, mwl, mdt, int(cigar), scores.ctypes.data, runs.ctypes.data if cigar else None,
            slot, nruns.ctypes.data, status.ctypes.data, threads, ctypes.byref(st))
    else:
        rc = lib.oracle_align_batch_ends(
            batch.patterns.ctypes.data, batch.p_off.ctypes.data, batch.p_len.ctypes.data,
            batch.texts.ctypes.data, batch.t_off.ctypes.data, batch.t_len.ctypes.data, N, x, o,
            e, pb, pe, tb, te, int(cigar), scores.ctypes.data,
            runs.ctypes.data if cigar else None, slot, nruns.ctypes.data, status.ctypes.data,
            threads, ctypes.byref(st))
    if rc != 0:
        raise RuntimeError(f"oracle_align_batch failed with status {rc}")
    bad = np.nonzero(status)[0]
    if bad.size:
        raise RuntimeError(f"oracle failed on pair {int(bad[0])} (status {int(status[bad[0]])}); "
                           f"raise `slot` above {int(nruns[bad[0]])}")
    offsets = np.zeros(N + 1, dtype=np.uint64)
    np.cumsum(nruns, out=offsets[1:])
    if cigar and N:
        keep = np.arange(slot)[None, :] < nruns[:, None]
        compact = runs.reshape(N, slot)[keep]
    else:
        compact = np.zeros(0, dtype=np.uint32)
    return BatchResult(scores, compact.astype(np.uint32), offsets, st.as_dict())


def pack2bit(seq: bytes) -> np.ndarray:
    """Packed words of one sequence (plain definition of the packed format)."""
    lib = _load()
    nwords = (len(seq) + 31) // 32
    words = np.zeros(max(nwords, 1), dtype=np.uint64)
    bad = lib.oracle_pack2bit(_buf(seq), len(seq), words.ctypes.data, nwords)
    if bad >= 0:
        raise ValueError(f"byte {bad} is not one of ACGT")
    return words[:nwords]


def cigar_string(runs) -> str:
    """Text form of runs: e.g. '48M1X51M'."""
    return "".join(f"{int(r) >> 4}{OP_CHARS[int(r) & 15]}" for r in runs)
