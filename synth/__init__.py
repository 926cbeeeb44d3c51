"""Seeded synthetic read pairs (input bytes only; no alignment arithmetic).

Shared by the CPU oracle's tests and the HIP library's tests and benchmark.
The generator itself is C (``synth.c``) so that millions of pairs are
produced in about a second; this module only marshals arrays.

Workload presets mirror the paper's experiment (Results: 5 million pairs of
100 bp reads at edit thresholds E = 2 % and 4 %) and the wider shapes used
to exercise the batching, long-read and serving paths.  The paper's own
read set is not public; these seeded generators stand in for it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")

LEN_FIXED, LEN_UNIFORM, LEN_LOGUNIFORM = 0, 1, 2
EDITS_FIXED, EDITS_RATE = 0, 1


class Spec(ctypes.Structure):
    _fields_ = [
        ("len_dist", ctypes.c_int32),
        ("n_lo", ctypes.c_uint32),
        ("n_hi", ctypes.c_uint32),
        ("edit_mode", ctypes.c_int32),
        ("edits", ctypes.c_uint32),
        ("r_lo", ctypes.c_double),
        ("r_hi", ctypes.c_double),
        ("runs", ctypes.c_int32),
    ]


def fixed(n: int, edits: int) -> Spec:
    """n-base patterns with exactly `edits` single-base edit events."""
    return Spec(LEN_FIXED, n, n, EDITS_FIXED, edits, 0.0, 0.0, 0)


def uneven(n_lo: int, n_hi: int, r_lo: float, r_hi: float) -> Spec:
    """Uniform lengths, per-pair edit rate uniform in [r_lo, r_hi)."""
    return Spec(LEN_UNIFORM, n_lo, n_hi, EDITS_RATE, 0, r_lo, r_hi, 0)


def long_reads(n_lo: int, n_hi: int, r_lo: float, r_hi: float) -> Spec:
    """Log-uniform lengths, event rate in [r_lo, r_hi), geometric indel runs."""
    return Spec(LEN_LOGUNIFORM, n_lo, n_hi, EDITS_RATE, 0, r_lo, r_hi, 1)


def loguniform_single(n_lo: int, n_hi: int, r_lo: float, r_hi: float) -> Spec:
    """Log-uniform lengths, per-pair rate, single-base events."""
    return Spec(LEN_LOGUNIFORM, n_lo, n_hi, EDITS_RATE, 0, r_lo, r_hi, 0)


# Named workloads: (spec, seed, default count)
WORKLOADS = {
    # 10k pairs of 100 bp, 2 edits (E = 2 %)
    "pairs100_e2_10k": (fixed(100, 2), 1, 10_000),
    # 5M pairs of 100 bp at E = 4 % and E = 2 %
    "pairs100_e4_5m": (fixed(100, 4), 2, 5_000_000),
    "pairs100_e2_5m": (fixed(100, 2), 3, 5_000_000),
    # 2M uneven pairs: 50-300 bp, 0-5 % edits
    "uneven50_300_2m": (uneven(50, 300, 0.0, 0.05), 4, 2_000_000),
    # 100k long pairs: 1-10 kbp log-uniform, 5-10 % events with indel runs
    "long1k_10k_100k": (long_reads(1000, 10000, 0.05, 0.10), 5, 100_000),
    # serving request bodies: 100-10,000 bp log-uniform, 1-10 % edits
    "serving_mix": (loguniform_single(100, 10000, 0.01, 0.10), 6, 0),
}

_lib = None


def build(force: bool = False) -> str:
    """Compile libsynth.so with the host C compiler."""
    src = os.path.join(_HERE, "synth.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        subprocess.check_call(
            ["gcc", "-O2", "-Wall", "-shared", "-fPIC", "-o", _LIB_PATH, src, "-lm"]
        )
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        p = ctypes.c_void_p
        lib.synth_lengths.argtypes = [ctypes.POINTER(Spec), ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.c_uint64, p, p]
        lib.synth_lengths.restype = ctypes.c_int
        lib.synth_fill.argtypes = [ctypes.POINTER(Spec), ctypes.c_uint64, ctypes.c_uint64,
                                   ctypes.c_uint64, p, p, p, p]
        lib.synth_fill.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Batch:
    """Concatenated ASCII sequences plus per-pair byte offsets and lengths."""

    patterns: np.ndarray  # uint8
    texts: np.ndarray  # uint8
    p_off: np.ndarray  # uint64
    p_len: np.ndarray  # uint32
    t_off: np.ndarray  # uint64
    t_len: np.ndarray  # uint32

    def __len__(self) -> int:
        return int(self.p_len.shape[0])

    def pair(self, i: int) -> tuple[bytes, bytes]:
        a = int(self.p_off[i])
        b = int(self.t_off[i])
        return (self.patterns[a:a + int(self.p_len[i])].tobytes(),
                self.texts[b:b + int(self.t_len[i])].tobytes())

    def subset(self, idx) -> "Batch":
        """A new, compacted batch holding the pairs at positions `idx`."""
        pairs = [self.pair(int(i)) for i in idx]
        return from_pairs(pairs)


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def generate(spec: Spec, seed: int, count: int, first: int = 0) -> Batch:
    """Pairs first .. first+count-1 of the stream defined by (spec, seed)."""
    lib = _load()
    p_len = np.zeros(count, dtype=np.uint32)
    t_len = np.zeros(count, dtype=np.uint32)
    if count:
        rc = lib.synth_lengths(ctypes.byref(spec), seed, first, count, _ptr(p_len), _ptr(t_len))
        if rc != 0:
            raise MemoryError("synth_lengths failed")
    p_off = np.zeros(count, dtype=np.uint64)
    t_off = np.zeros(count, dtype=np.uint64)
    if count > 1:
        np.cumsum(p_len[:-1], dtype=np.uint64, out=p_off[1:])
        np.cumsum(t_len[:-1], dtype=np.uint64, out=t_off[1:])
    pbuf = np.zeros(int(p_len.sum(dtype=np.uint64)) + 1, dtype=np.uint8)
    tbuf = np.zeros(int(t_len.sum(dtype=np.uint64)) + 1, dtype=np.uint8)
    if count:
        rc = lib.synth_fill(ctypes.byref(spec), seed, first, count, _ptr(p_off), _ptr(t_off),
                            _ptr(pbuf), _ptr(tbuf))
        if rc != 0:
            raise MemoryError("synth_fill failed")
    return Batch(pbuf, tbuf, p_off, p_len, t_off, t_len)


def workload(name: str, count: int | None = None, first: int = 0) -> Batch:
    spec, seed, default = WORKLOADS[name]
    return generate(spec, seed, default if count is None else count, first)


def from_pairs(pairs) -> Batch:
    """Pack explicit (pattern, text) byte strings into a Batch."""
    pats = [bytes(p) for p, _ in pairs]
    txts = [bytes(t) for _, t in pairs]
    p_len = np.array([len(p) for p in pats], dtype=np.uint32)
    t_len = np.array([len(t) for t in txts], dtype=np.uint32)
    p_off = np.zeros(len(pats), dtype=np.uint64)
    t_off = np.zeros(len(txts), dtype=np.uint64)
    if len(pats) > 1:
        np.cumsum(p_len[:-1], dtype=np.uint64, out=p_off[1:])
        np.cumsum(t_len[:-1], dtype=np.uint64, out=t_off[1:])
    pbuf = np.frombuffer(b"".join(pats) + b"\0", dtype=np.uint8).copy()
    tbuf = np.frombuffer(b"".join(txts) + b"\0", dtype=np.uint8).copy()
    return Batch(pbuf, tbuf, p_off, p_len, t_off, t_len)


def random_pairs(rng: np.random.Generator, count: int, n_max: int, alphabet: bytes = b"ACGT",
                 related: bool = True):
    """Small unrelated or mutated pairs for property tests (numpy RNG)."""
    out = []
    for _ in range(count):
        n = int(rng.integers(0, n_max + 1))
        p = bytes(rng.choice(list(alphabet), size=n).astype(np.uint8)) if n else b""
        if related and n:
            t = bytearray(p)
            for _ in range(int(rng.integers(0, max(1, n // 3) + 1))):
                op = int(rng.integers(0, 3))
                pos = int(rng.integers(0, len(t) + 1))
                b = alphabet[int(rng.integers(0, len(alphabet)))]
                if op == 0 and pos < len(t):
                    t[pos] = b
                elif op == 1:
                    t.insert(pos, b)
                elif pos < len(t):
                    del t[pos]
            t = bytes(t)
        else:
            m = int(rng.integers(0, n_max + 1))
            t = bytes(rng.choice(list(alphabet), size=m).astype(np.uint8)) if m else b""
        out.append((p, t))
    return out
