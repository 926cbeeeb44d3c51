"""Independent references that pin the oracle (plain Python, no WFA).

* ``enumerate_costs``: every global alignment of two tiny strings, scored
  directly from the gap-affine definition (pins the dynamic programs).
* ``gotoh``: the textbook three-state dynamic program (Gotoh 1982) with
  co-optimal alignment counting and a traceback of one optimum.
* ``gotoh_np``: the same recurrences row by row in numpy for longer pairs
  (the row-wise insertion minimum uses a running prefix minimum).
* ``levenshtein``: the unit-cost edit distance (Wagner-Fischer).
* ``check_cigar``: spells both sequences from a CIGAR and re-scores it.

The affine cost model: mismatch x, a gap of length L costs o + L*e, matches
cost 0.  None of this code calls or mirrors the oracle.
"""
from __future__ import annotations

import numpy as np

INF = float("inf")
OP_M, OP_X, OP_I, OP_D = 0, 1, 2, 3


def alignment_cost(P: bytes, T: bytes, ops: str, x: int, o: int, e: int) -> int:
    """Cost of an op string over 'MXID' (M/X both diagonal; checked vs bases)."""
    v = h = 0
    cost = 0
    prev = None
    for op in ops:
        if op in "MX":
            cost += 0 if P[v] == T[h] else x
            v += 1
            h += 1
        elif op == "I":
            cost += e + (o if prev != "I" else 0)
            h += 1
        else:
            cost += e + (o if prev != "D" else 0)
            v += 1
        prev = op
    assert v == len(P) and h == len(T)
    return cost


def enumerate_alignments(n: int, m: int):
    """All op strings ('M' diagonal, 'I' text-only, 'D' pattern-only)."""
    if n == 0 and m == 0:
        yield ""
        return
    if n > 0 and m > 0:
        for rest in enumerate_alignments(n - 1, m - 1):
            yield "M" + rest
    if m > 0:
        for rest in enumerate_alignments(n, m - 1):
            yield "I" + rest
    if n > 0:
        for rest in enumerate_alignments(n - 1, m):
            yield "D" + rest


def enumerate_costs(P: bytes, T: bytes, x: int, o: int, e: int):
    """(min cost, number of optimal alignments) by exhaustive enumeration."""
    best = INF
    count = 0
    for ops in enumerate_alignments(len(P), len(T)):
        c = alignment_cost(P, T, ops, x, o, e)
        if c < best:
            best, count = c, 1
        elif c == best:
            count += 1
    return int(best), count


def gotoh(P: bytes, T: bytes, x: int, o: int, e: int, traceback: bool = False):
    """Three-state affine DP.

    States: Dg[v][h] = best cost of aligning P[:v], T[:h] ending with a
    diagonal column; Ig ending with a text-only column; Dl ending with a
    pattern-only column.  Each alignment is exactly one state path, so
    counting optimal paths counts optimal alignments.

    Returns (score, count) or (score, count, ops) where ops is the op string
    of one optimal alignment ('M' match, 'X' mismatch, 'I', 'D').
    """
    n, m = len(P), len(T)
    Dg = [[INF] * (m + 1) for _ in range(n + 1)]
    Ig = [[INF] * (m + 1) for _ in range(n + 1)]
    Dl = [[INF] * (m + 1) for _ in range(n + 1)]
    cD = [[0] * (m + 1) for _ in range(n + 1)]
    cI = [[0] * (m + 1) for _ in range(n + 1)]
    cL = [[0] * (m + 1) for _ in range(n + 1)]
    Dg[0][0] = 0
    cD[0][0] = 1  # the empty alignment, counted once through the diagonal state
    for v in range(n + 1):
        for h in range(m + 1):
            if v > 0 and h > 0:
                sub = 0 if P[v - 1] == T[h - 1] else x
                cands = [(Dg[v - 1][h - 1], cD[v - 1][h - 1]), (Ig[v - 1][h - 1], cI[v - 1][h - 1]),
                         (Dl[v - 1][h - 1], cL[v - 1][h - 1])]
                b = min(c for c, _ in cands)
                if b < INF:
                    Dg[v][h] = b + sub
                    cD[v][h] = sum(k for c, k in cands if c == b)
            if h > 0:
                cands = [(Dg[v][h - 1] + o + e, cD[v][h - 1]), (Ig[v][h - 1] + e, cI[v][h - 1]),
                         (Dl[v][h - 1] + o + e, cL[v][h - 1])]
                b = min(c for c, _ in cands)
                if b < INF:
                    Ig[v][h] = b
                    cI[v][h] = sum(k for c, k in cands if c == b)
            if v > 0:
                cands = [(Dg[v - 1][h] + o + e, cD[v - 1][h]), (Ig[v - 1][h] + o + e, cI[v - 1][h]),
                         (Dl[v - 1][h] + e, cL[v - 1][h])]
                b = min(c for c, _ in cands)
                if b < INF:
                    Dl[v][h] = b
                    cL[v][h] = sum(k for c, k in cands if c == b)
    final = [(Dg[n][m], cD[n][m]), (Ig[n][m], cI[n][m]), (Dl[n][m], cL[n][m])]
    score = min(c for c, _ in final)
    count = sum(k for c, k in final if c == score)
    if not traceback:
        return int(score), count
    # walk back one optimal path
    ops = []
    v, h = n, m
    state = min(range(3), key=lambda i: final[i][0])
    tables = (Dg, Ig, Dl)
    while v > 0 or h > 0:
        cur = tables[state][v][h]
        if state == 0:
            sub = 0 if P[v - 1] == T[h - 1] else x
            ops.append("M" if sub == 0 else "X")
            prev = [Dg[v - 1][h - 1], Ig[v - 1][h - 1], Dl[v - 1][h - 1]]
            state = next(i for i in range(3) if prev[i] + sub == cur)
            v, h = v - 1, h - 1
        elif state == 1:
            ops.append("I")
            prev = [Dg[v][h - 1] + o + e, Ig[v][h - 1] + e, Dl[v][h - 1] + o + e]
            state = next(i for i in range(3) if prev[i] == cur)
            h -= 1
        else:
            ops.append("D")
            prev = [Dg[v - 1][h] + o + e, Ig[v - 1][h] + o + e, Dl[v - 1][h] + e]
            state = next(i for i in range(3) if prev[i] == cur)
            v -= 1
    return int(score), count, "".join(reversed(ops))


def gotoh_np(P: bytes, T: bytes, x: int, o: int, e: int) -> int:
    """Gotoh score, one row at a time in numpy (int64, big sentinel)."""
    n, m = len(P), len(T)
    BIG = 1 << 40
    p = np.frombuffer(P, dtype=np.uint8)
    t = np.frombuffer(T, dtype=np.uint8)
    hh = np.arange(m + 1, dtype=np.int64)
    # row 0
    H = np.where(hh == 0, 0, o + hh * e)  # best of any state
    D = np.full(m + 1, BIG, dtype=np.int64)  # ending with a pattern-only column
    for v in range(1, n + 1):
        # D from the row above
        D = np.minimum(D + e, H + o + e)
        # diagonal
        diag = np.full(m + 1, BIG, dtype=np.int64)
        diag[1:] = H[:-1] + np.where(p[v - 1] == t, 0, x)
        base = np.minimum(diag, D)
        base[0] = min(D[0], BIG)
        # I[h] = min over h' < h of base[h'] + o + (h - h') e  (row-internal gaps)
        key = base - hh * e
        run = np.minimum.accumulate(key)
        I = np.full(m + 1, BIG, dtype=np.int64)
        I[1:] = run[:-1] + o + hh[1:] * e
        H = np.minimum(base, I)
    return int(H[m])


def levenshtein(P: bytes, T: bytes) -> int:
    n, m = len(P), len(T)
    prev = list(range(m + 1))
    for v in range(1, n + 1):
        cur = [v] + [0] * m
        for h in range(1, m + 1):
            cur[h] = min(prev[h] + 1, cur[h - 1] + 1, prev[h - 1] + (P[v - 1] != T[h - 1]))
        prev = cur
    return prev[m]


def runs_to_ops(runs) -> str:
    return "".join("MXID"[int(r) & 15] * (int(r) >> 4) for r in runs)


def check_cigar(P: bytes, T: bytes, runs, x: int, o: int, e: int):
    """Validate a run list against both sequences; return its affine cost.

    Raises AssertionError if the runs do not spell P and T, if an M column
    holds different bases or an X column equal ones, if a run is empty or
    two neighbouring runs share an op.
    """
    prev_op = None
    for r in runs:
        assert int(r) >> 4 > 0, "empty run"
        assert (int(r) & 15) < 4, "bad op code"
        assert (int(r) & 15) != prev_op, "runs not maximal"
        prev_op = int(r) & 15
    ops = runs_to_ops(runs)
    v = h = 0
    for op in ops:
        if op == "M":
            assert v < len(P) and h < len(T) and P[v] == T[h], f"M on mismatch at {v},{h}"
            v += 1
            h += 1
        elif op == "X":
            assert v < len(P) and h < len(T) and P[v] != T[h], f"X on match at {v},{h}"
            v += 1
            h += 1
        elif op == "I":
            assert h < len(T)
            h += 1
        else:
            assert v < len(P)
            v += 1
    assert v == len(P) and h == len(T), "CIGAR does not consume both sequences"
    return alignment_cost(P, T, ops, x, o, e)


# ---- ends-free alignment ------------------------------------------------------
# At most pb leading / pe trailing pattern bases, or tb leading / te trailing
# text bases, may stay unaligned at no cost; `ends` = (pb, pe, tb, te), each
# clipped to its sequence's length.  (0, 0, 0, 0) is global alignment.

def _clip_ends(n: int, m: int, ends):
    pb, pe, tb, te = ends
    return min(pb, n), min(pe, n), min(tb, m), min(te, m)


def ends_free_by_subpairs(P: bytes, T: bytes, x: int, o: int, e: int, ends, global_score):
    """The definition written out: the least global score, over every allowed
    start (v, 0) with v <= pb or (0, h) with h <= tb and every allowed end
    (v, m) with v >= n - pe or (n, h) with h >= m - te, of the pair clipped
    to that start and end.  `global_score(P, T, x, o, e)` scores a pair."""
    n, m = len(P), len(T)
    pb, pe, tb, te = _clip_ends(n, m, ends)
    starts = {(v, 0) for v in range(pb + 1)} | {(0, h) for h in range(tb + 1)}
    stops = {(v, m) for v in range(n - pe, n + 1)} | {(n, h) for h in range(m - te, m + 1)}
    best = INF
    for vb, hb in starts:
        for ve, he in stops:
            if ve >= vb and he >= hb:
                best = min(best, global_score(P[vb:ve], T[hb:he], x, o, e))
    return int(best)


def gotoh_ends(P: bytes, T: bytes, x: int, o: int, e: int, ends) -> int:
    """Gotoh's three-state DP with free boundary cells: every allowed start
    cell holds cost 0 in the diagonal state (a fresh start: a gap after it
    opens), and the score is the least cost over the allowed end cells."""
    n, m = len(P), len(T)
    pb, pe, tb, te = _clip_ends(n, m, ends)
    Dg = [[INF] * (m + 1) for _ in range(n + 1)]
    Ig = [[INF] * (m + 1) for _ in range(n + 1)]
    Dl = [[INF] * (m + 1) for _ in range(n + 1)]
    for v in range(n + 1):
        for h in range(m + 1):
            if (v == 0 and h <= tb) or (h == 0 and v <= pb):
                Dg[v][h] = 0
            if v > 0 and h > 0:
                sub = 0 if P[v - 1] == T[h - 1] else x
                Dg[v][h] = min(Dg[v][h],
                               min(Dg[v - 1][h - 1], Ig[v - 1][h - 1], Dl[v - 1][h - 1]) + sub)
            if h > 0:
                Ig[v][h] = min(Dg[v][h - 1] + o + e, Ig[v][h - 1] + e, Dl[v][h - 1] + o + e)
            if v > 0:
                Dl[v][h] = min(Dg[v - 1][h] + o + e, Ig[v - 1][h] + o + e, Dl[v - 1][h] + e)
    cells = {(v, m) for v in range(n - pe, n + 1)} | {(n, h) for h in range(m - te, m + 1)}
    return int(min(min(Dg[v][h], Ig[v][h], Dl[v][h]) for v, h in cells))


def check_cigar_ends(P: bytes, T: bytes, runs, x: int, o: int, e: int, ends) -> int:
    """Validate a run list against both sequences (as check_cigar) and return
    its ends-free cost: a leading I (D) run is free for up to tb (pb) bases,
    a trailing I (D) run for up to te (pe) bases, and what is left of such a
    run is an ordinary gap."""
    check_cigar(P, T, runs, 0, 0, 1)  # spelling and run rules only
    n, m = len(P), len(T)
    pb, pe, tb, te = _clip_ends(n, m, ends)
    ops = runs_to_ops(runs)
    vb = hb = 0
    lead = len(ops) - len(ops.lstrip(ops[:1])) if ops else 0
    if ops[:1] == "I":
        hb = min(lead, tb)
    elif ops[:1] == "D":
        vb = min(lead, pb)
    ops = ops[hb + vb:]
    ve, he = n, m
    trail = len(ops) - len(ops.rstrip(ops[-1:])) if ops else 0
    if ops[-1:] == "I":
        he = m - min(trail, te)
    elif ops[-1:] == "D":
        ve = n - min(trail, pe)
    ops = ops[: len(ops) - (n - ve) - (m - he)]
    return alignment_cost(P[vb:ve], T[hb:he], ops, x, o, e)
