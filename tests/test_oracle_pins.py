"""Pins for the CPU oracle: each test ties it to something other than itself.

* closed forms (tests/golden/closed_forms.tsv),
* exhaustive enumeration of all alignments (pins the Gotoh DP),
* the textbook Gotoh DP on every pair of short strings and on random
  longer pairs,
* the Levenshtein special case (x, o, e) = (1, 0, 1),
* CIGAR invariants (spells both sequences, M/X are true matches and
  mismatches, re-scores to the reported optimum),
* equality with the Gotoh traceback where the optimum is unique,
* symmetry and the planted-edit upper bound on generated read pairs,
* ends-free alignment: the definition (least global score over the allowed
  clipped sub-pairs) by enumeration and by the pinned Gotoh DP, a Gotoh DP
  with free boundary cells, closed forms (semi-global, overlaps) and the
  symmetry of swapping the sequences,
* the WF-adaptive heuristic: a worked example derived by hand from the
  reduction's definition (both sides of the width and threshold
  comparisons), exactness where no reduction can act, and that every result
  is an alignment scoring at least the optimum,
* planted mistakes: mutants of the oracle built on the CPU must fail the
  pins above.
"""
import itertools
import os
import subprocess

import numpy as np
import pytest

import brute

HERE = os.path.dirname(os.path.abspath(__file__))
PENALTIES = [(4, 6, 2), (1, 0, 1), (2, 3, 1), (3, 1, 4), (5, 7, 1), (1, 5, 1), (7, 2, 3)]


def strings(alphabet: bytes, max_len: int):
    for L in range(max_len + 1):
        for t in itertools.product(alphabet, repeat=L):
            yield bytes(t)


def load_golden():
    rows = []
    with open(os.path.join(HERE, "golden", "closed_forms.tsv")) as f:
        for line in f:
            if line.startswith("#") or line.startswith("pattern\t") or not line.strip():
                continue
            p, t, x, o, e, score, cigar, why = line.rstrip("\n").split("\t")
            p = b"" if p == "-" else p.encode()
            t = b"" if t == "-" else t.encode()
            rows.append((p, t, (int(x), int(o), int(e)), int(score), cigar, why))
    return rows


@pytest.mark.parametrize("row", load_golden(), ids=lambda r: r[5][:40])
def test_golden_closed_forms(oracle_lib, row):
    p, t, pen, score, cigar, _ = row
    s, runs = oracle_lib.align(p, t, pen)
    assert s == score
    if cigar != "*":
        assert oracle_lib.cigar_string(runs) == ("" if cigar == "-" else cigar)
    assert brute.check_cigar(p, t, runs, *pen) == score
    # the closed form also holds for the independent DP
    assert brute.gotoh(p, t, *pen)[0] == score


def test_enumeration_pins_gotoh():
    """Gotoh's score and co-optimal count equal exhaustive enumeration."""
    pairs = list(itertools.product(list(strings(b"ACGT", 3)), repeat=2))
    pairs += list(itertools.product([s for s in strings(b"AC", 4) if len(s) == 4], repeat=2))
    for pen in [(4, 6, 2), (1, 0, 1), (3, 1, 4), (20, 1, 1)]:
        for p, t in pairs:
            assert brute.gotoh(p, t, *pen) == brute.enumerate_costs(p, t, *pen), (p, t, pen)


def test_gotoh_np_matches_plain_gotoh():
    rng = np.random.default_rng(11)
    for pen in PENALTIES:
        for p, t in [(b"", b""), (b"", b"AC"), (b"GT", b"")] + [
                (bytes(rng.choice(list(b"ACGT"), int(rng.integers(0, 25))).astype(np.uint8)),
                 bytes(rng.choice(list(b"ACGT"), int(rng.integers(0, 25))).astype(np.uint8)))
                for _ in range(40)]:
            assert brute.gotoh_np(p, t, *pen) == brute.gotoh(p, t, *pen)[0]


@pytest.mark.parametrize("pen", PENALTIES)
def test_oracle_exhaustive_short(oracle_lib, pen):
    """Every pair over ACGT up to length 3 and over AC up to length 5."""
    seqs = list(strings(b"ACGT", 3)) + [s for s in strings(b"AC", 5) if len(s) >= 4]
    for p, t in itertools.product(seqs, repeat=2):
        s, runs = oracle_lib.align(p, t, pen)
        g, count, ops = brute.gotoh(p, t, *pen, traceback=True)
        assert s == g, (p, t, pen)
        assert brute.check_cigar(p, t, runs, *pen) == s
        if count == 1:
            assert brute.runs_to_ops(runs) == ops, (p, t, pen)


@pytest.mark.parametrize("pen", PENALTIES)
def test_oracle_random_vs_gotoh(oracle_lib, synth_lib, pen):
    rng = np.random.default_rng(1234 + sum(pen))
    pairs = synth_lib.random_pairs(rng, 60, 120) + synth_lib.random_pairs(rng, 10, 300)
    pairs += synth_lib.random_pairs(rng, 10, 60, related=False)
    for p, t in pairs:
        s, runs = oracle_lib.align(p, t, pen)
        assert s == brute.gotoh_np(p, t, *pen), (p, t, pen)
        assert brute.check_cigar(p, t, runs, *pen) == s
        s2, _ = oracle_lib.align(t, p, pen, cigar=False)
        assert s2 == s  # symmetry of the affine score


def test_oracle_unique_optimum_cigar(oracle_lib, synth_lib):
    """Where Gotoh finds exactly one optimal alignment the CIGAR is fixed."""
    rng = np.random.default_rng(77)
    checked = 0
    for p, t in synth_lib.random_pairs(rng, 300, 40):
        for pen in [(4, 6, 2), (5, 7, 1)]:
            g, count, ops = brute.gotoh(p, t, *pen, traceback=True)
            if count != 1:
                continue
            s, runs = oracle_lib.align(p, t, pen)
            assert s == g
            assert brute.runs_to_ops(runs) == ops, (p, t, pen)
            checked += 1
    assert checked > 100


def test_levenshtein_special_case(oracle_lib, synth_lib):
    rng = np.random.default_rng(5)
    for p, t in synth_lib.random_pairs(rng, 80, 80) + synth_lib.random_pairs(rng, 20, 40, related=False):
        s, runs = oracle_lib.align(p, t, (1, 0, 1))
        assert s == brute.levenshtein(p, t)
        assert brute.check_cigar(p, t, runs, 1, 0, 1) == s


def test_score_only_equals_cigar_mode(oracle_lib, synth_lib):
    b = synth_lib.workload("uneven50_300_2m", 300)
    for pen in [(4, 6, 2), (2, 3, 1)]:
        full = oracle_lib.align_batch(b, pen, cigar=True, threads=4)
        sc = oracle_lib.align_batch(b, pen, cigar=False, threads=4)
        assert np.array_equal(full.scores, sc.scores)


def test_generated_pairs_properties(oracle_lib, synth_lib):
    """Planted-edit bound and CIGAR invariants on the 100 bp workloads."""
    x, o, e = 4, 6, 2
    for name, edits in [("pairs100_e2_10k", 2), ("pairs100_e4_5m", 4)]:
        b = synth_lib.workload(name, 400)
        r = oracle_lib.align_batch(b, (x, o, e), threads=4)
        # every planted event costs at most o + e (indel) or x (substitution)
        assert int(r.scores.max()) <= edits * max(x, o + e)
        assert int(r.scores.min()) >= 0
        for i in range(len(b)):
            p, t = b.pair(i)
            runs = r.runs[int(r.offsets[i]):int(r.offsets[i + 1])]
            assert brute.check_cigar(p, t, runs, x, o, e) == int(r.scores[i])
        for i in range(0, len(b), 37):
            p, t = b.pair(i)
            assert brute.gotoh_np(p, t, x, o, e) == int(r.scores[i])


def test_batch_equals_single(oracle_lib, synth_lib):
    b = synth_lib.workload("uneven50_300_2m", 64)
    r = oracle_lib.align_batch(b, (4, 6, 2), threads=3)
    for i in range(len(b)):
        s, runs = oracle_lib.align(*b.pair(i), (4, 6, 2))
        assert s == int(r.scores[i])
        assert list(r.runs[int(r.offsets[i]):int(r.offsets[i + 1])]) == runs


def test_pack2bit_definition(oracle_lib):
    # A=0 C=1 G=2 T=3, base i at bits 2*(i%32) of word i//32
    w = oracle_lib.pack2bit(b"ACGT")
    assert w.tolist() == [0 | 1 << 2 | 2 << 4 | 3 << 6]
    w = oracle_lib.pack2bit(b"T" * 33)
    assert w.tolist() == [(1 << 64) - 1, 3]
    assert oracle_lib.pack2bit(b"acgt").tolist() == oracle_lib.pack2bit(b"ACGT").tolist()
    with pytest.raises(ValueError):
        oracle_lib.pack2bit(b"ACNT")


# ---- ends-free alignment -----------------------------------------------------
# (pattern_begin_free, pattern_end_free, text_begin_free, text_end_free)
ENDS_SHORT = [(1, 0, 0, 1), (0, 2, 2, 0), (3, 3, 3, 3), (0, 0, 9, 9), (9, 9, 0, 0), (1, 2, 0, 0)]


def _gotoh_score(P, T, x, o, e):
    return brute.gotoh(P, T, x, o, e)[0]


def _enum_score(P, T, x, o, e):
    return brute.enumerate_costs(P, T, x, o, e)[0]


@pytest.mark.parametrize("ends", ENDS_SHORT)
def test_ends_free_exhaustive_short(oracle_lib, ends):
    """Every pair of strings over {A, C} of up to 3 bases: the oracle's
    ends-free score is the definition's (least global score over the
    allowed starts and ends, each global score by the pinned Gotoh DP), and
    its CIGAR spells both sequences and re-scores to it."""
    for pen in [(4, 6, 2), (1, 0, 1), (3, 1, 4)]:
        for P in strings(b"AC", 3):
            for T in strings(b"AC", 3):
                s, runs = oracle_lib.align(P, T, pen, ends=ends)
                assert s == brute.ends_free_by_subpairs(P, T, *pen, ends, _gotoh_score), (P, T)
                assert brute.check_cigar_ends(P, T, runs, *pen, ends) == s, (P, T, runs)


def test_ends_free_dp_matches_definition():
    """The free-boundary DP equals the definition evaluated by exhaustive
    enumeration of alignments (no DP) on random tiny pairs."""
    rng = np.random.default_rng(17)
    for _ in range(150):
        P = bytes(rng.choice(list(b"ACG"), int(rng.integers(0, 5))).astype(np.uint8))
        T = bytes(rng.choice(list(b"ACG"), int(rng.integers(0, 5))).astype(np.uint8))
        ends = tuple(int(v) for v in rng.integers(0, 5, 4))
        pen = PENALTIES[int(rng.integers(0, len(PENALTIES)))]
        assert brute.gotoh_ends(P, T, *pen, ends) == brute.ends_free_by_subpairs(
            P, T, *pen, ends, _enum_score), (P, T, pen, ends)


@pytest.mark.parametrize("pen", [(4, 6, 2), (1, 0, 1), (2, 3, 1), (7, 2, 3)])
def test_ends_free_random_vs_dp(oracle_lib, synth_lib, pen):
    """Random related pairs of up to 40 bases with random free ends: score
    equal to the free-boundary DP, CIGAR re-scores to it; all-zero ends give
    the global alignment exactly (score and CIGAR)."""
    rng = np.random.default_rng(hash(pen) % 1000)
    for P, T in synth_lib.random_pairs(rng, 60, 40):
        ends = tuple(int(v) for v in rng.integers(0, 12, 4))
        s, runs = oracle_lib.align(P, T, pen, ends=ends)
        assert s == brute.gotoh_ends(P, T, *pen, ends), (P, T, ends)
        assert brute.check_cigar_ends(P, T, runs, *pen, ends) == s
        assert oracle_lib.align(P, T, pen, ends=(0, 0, 0, 0)) == oracle_lib.align(P, T, pen)


def test_ends_free_closed_forms(oracle_lib):
    """Semi-global and overlap cases whose answer is known outright."""
    T = b"GGATTACACCGT"
    # the pattern occurs in the text: free text ends cost nothing
    s, runs = oracle_lib.align(b"TTACA", T, ends=(0, 0, len(T), len(T)))
    assert s == 0 and oracle_lib.cigar_string(runs) == "3I5M4I"
    # a free text prefix shorter than the offset: the rest is a paid gap
    s, runs = oracle_lib.align(b"TTACA", b"GGATTACA", ends=(0, 0, 1, 0))
    assert s == 6 + 2 * 2 and oracle_lib.cigar_string(runs) == "3I5M"
    # suffix of the pattern overlaps a prefix of the text
    s, runs = oracle_lib.align(b"CCCCACGT", b"ACGTGGGG", ends=(4, 0, 0, 4))
    assert s == 0 and oracle_lib.cigar_string(runs) == "4D4M4I"
    # free ends on both sides of an empty pattern
    s, runs = oracle_lib.align(b"", b"ACGT", ends=(0, 0, 2, 2))
    assert s == 0 and oracle_lib.cigar_string(runs) == "4I"
    s, runs = oracle_lib.align(b"", b"ACGTA", ends=(0, 0, 2, 2))
    assert s == 6 + 2 and oracle_lib.cigar_string(runs) == "5I"
    # symmetry: swapping the sequences swaps the free pattern and text ends
    rng = np.random.default_rng(5)
    for P, T in [(bytes(rng.choice(list(b"ACGT"), 25).astype(np.uint8)),
                  bytes(rng.choice(list(b"ACGT"), 31).astype(np.uint8))) for _ in range(30)]:
        for pb, pe, tb, te in [(3, 0, 0, 5), (0, 7, 2, 0), (4, 4, 4, 4)]:
            a = oracle_lib.align(P, T, ends=(pb, pe, tb, te))[0]
            b = oracle_lib.align(T, P, ends=(tb, te, pb, pe))[0]
            assert a == b


# ---- WF-adaptive heuristic ---------------------------------------------------
# Worked by hand from the reduction's definition, penalties (4, 6, 2),
# P = AA (n = 2), T = CCAA (m = 4); the optimum inserts CC (score 10, 2I2M).
#  s=0  k=0 holds h=0 (A/C mismatch), distance max(2-0, 4-0) = 4.
#  s=2  span [-1, 1], no offset (only gap extensions could reach it).
#  s=4  X: k=0, h=1 (A/C mismatch again), distance 3; span [-2, 2] of width
#       5; the reduction keeps [0, 0] once 5 >= min_wavefront_length.
#  s=6  span [-2, 2] (from s=2 and s=4, one diagonal wider), no offset.
#  s=8  span [-3, 3], width 7.  X: k=0, h=2 (v=2=n), distance max(0, 2) = 2;
#       I opened from s=0: k=1, h=1, no match, distance max(2, 3) = 3;
#       D opened from s=0: k=-1, h=0, distance max(1, 4) = 4.
#       With the threshold 0 only k=0 stays, and the 2I path (which needs
#       the I cell at k=1) is lost; threshold 1 keeps k=1 (3 <= 2 + 1).
#  Threshold 0 then ends at s=14: I opened at s=12 from (v, h) = (1, 1),
#  extended at s=14, one match: 1X2I1M, 4 + 6 + 2 + 2 = 14.  The reduction
#  first bites at s=8 (width 7), unless s=4 (width 5) already trimmed: any
#  min_wavefront_length up to 7 gives 14; from 8 on, no wavefront before the
#  end reaches the width (s=10 spans [-2, 4] after clipping: 7) and the
#  result is the exact one.  Swapping the sequences turns I into D.
# Distances are taken after the extension: P = AC, T = CAC (optimum 1I2M, 8)
# with (1, 0).  s=0: k=0, h=0, distance 3; s=4: X to k=0, h=1 (C/A), distance
# 2, kept alone; s=8: X to k=0, h=2 (v = n), distance 1; I from s=0 to k=1,
# h=1, which extends over AC to the end cell (h = 3): score 8.  Measured
# before the extension that I cell would sit at distance 2 and be dropped.
ADAPTIVE_WORKED = [
    (b"AC", b"CAC", (1, 0), 8, "1I2M"),
    (b"AA", b"CCAA", (1, 0), 14, "1X2I1M"),
    (b"AA", b"CCAA", (5, 0), 14, "1X2I1M"),
    (b"AA", b"CCAA", (7, 0), 14, "1X2I1M"),
    (b"AA", b"CCAA", (8, 0), 10, "2I2M"),
    (b"AA", b"CCAA", (1, 1), 10, "2I2M"),
    (b"AA", b"CCAA", (0, 0), 10, "2I2M"),
    (b"CCAA", b"AA", (1, 0), 14, "1X2D1M"),
    (b"CCAA", b"AA", (1, 1), 10, "2D2M"),
]


def test_adaptive_worked_example(oracle_lib):
    for P, T, ad, score, cigar in ADAPTIVE_WORKED:
        s, runs = oracle_lib.align(P, T, (4, 6, 2), adaptive=ad)
        assert (s, oracle_lib.cigar_string(runs)) == (score, cigar), (P, T, ad)
        assert brute.check_cigar(P, T, runs, 4, 6, 2) == s


def _adaptive_cases(synth_lib, seed):
    rng = np.random.default_rng(seed)
    pairs = synth_lib.random_pairs(rng, 40, 80) + synth_lib.random_pairs(rng, 10, 200)
    pairs += synth_lib.random_pairs(rng, 10, 40, related=False)
    pairs += [(b"", b""), (b"", b"ACG"), (b"GT", b""), (b"A", b"A")]
    return pairs


@pytest.mark.parametrize("pen", [(4, 6, 2), (1, 0, 1), (2, 3, 1)])
def test_adaptive_without_reduction_is_exact(oracle_lib, synth_lib, pen):
    """No reduction can happen when no wavefront reaches the minimum width
    (longer than any span: n + m + 2), and none changes a result when the
    threshold covers every distance (max(n, m)): both give the Gotoh
    optimum."""
    for P, T in _adaptive_cases(synth_lib, 31 + sum(pen)):
        g = brute.gotoh_np(P, T, *pen)
        n, m = len(P), len(T)
        assert oracle_lib.align(P, T, pen, adaptive=(n + m + 2, 0)) == oracle_lib.align(P, T, pen)
        s, runs = oracle_lib.align(P, T, pen, adaptive=(1, max(n, m)))
        assert s == g, (P, T)
        assert brute.check_cigar(P, T, runs, *pen) == s


@pytest.mark.parametrize("ad", [(1, 0), (3, 1), (10, 5), (10, 50), (20, 2)])
def test_adaptive_results_are_alignments(oracle_lib, synth_lib, ad):
    """Whatever it drops, the heuristic reports an alignment: its CIGAR
    spells both sequences and costs between the optimum and the reported
    score, the score of the path the search took (the path may close a gap
    and open one of the same kind at once, which the CIGAR writes as one
    run, one opening cheaper); score-only mode agrees with CIGAR mode."""
    below = cheaper = 0
    for P, T in _adaptive_cases(synth_lib, 7 + ad[0]):
        for pen in [(4, 6, 2), (1, 0, 1), (2, 3, 1)]:
            s, runs = oracle_lib.align(P, T, pen, adaptive=ad)
            g = brute.gotoh_np(P, T, *pen)
            c = brute.check_cigar(P, T, runs, *pen)
            assert g <= c <= s, (P, T, pen)
            below += s > g
            cheaper += c < s
            assert oracle_lib.align(P, T, pen, cigar=False, adaptive=ad)[0] == s
    if ad[1] <= 1:
        assert below > 0  # tight thresholds do lose the optimum somewhere
    assert cheaper <= below


def test_adaptive_reopened_gap():
    """A path that reopens a gap right after closing it: with (2, 3, 1) and
    (1, 0) the search reaches the end at 51 along a path whose CIGAR, with
    the two deletions merged into one run, costs 48 (one opening less)."""
    import oracle
    import synth

    rng = np.random.default_rng(37)
    pairs = synth.random_pairs(rng, 300, 120) + synth.random_pairs(rng, 60, 300)
    P, T = pairs[344]
    s, runs = oracle.align(P, T, (2, 3, 1), adaptive=(1, 0))
    assert s == 51 and brute.check_cigar(P, T, runs, 2, 3, 1) == 48
    assert brute.gotoh_np(P, T, 2, 3, 1) <= 48


def test_adaptive_batch_equals_single(oracle_lib, synth_lib):
    b = synth_lib.workload("uneven50_300_2m", 48)
    r = oracle_lib.align_batch(b, (4, 6, 2), threads=3, adaptive=(5, 3))
    for i in range(len(b)):
        s, runs = oracle_lib.align(*b.pair(i), (4, 6, 2), adaptive=(5, 3))
        assert s == int(r.scores[i])
        assert list(r.runs[int(r.offsets[i]):int(r.offsets[i + 1])]) == runs


# ---- the oracle's work counters --------------------------------------------
# The benchmark's algorithmic work per pair (cells, 32-base extension
# windows) comes from the oracle's counters, so they are pinned too, by
# closed forms that follow from the method's definitions:
#  * a wavefront at score s spans one diagonal more on each side than the
#    widest of its source wavefronts (s - x, s - o - e, s - e), clipped to
#    [-n, m].  Under (4, 6, 2) every even score has a wavefront (s - 2 always
#    does), so the span at s is [-s/2, s/2]: s + 1 cells, and a pair of score
#    S (with S/2 <= min(n, m)) visits 1 + 3 + ... + (S + 1) = (S/2 + 1)^2
#    cells in S/2 + 1 steps.  Under (1, 0, 1) every score has one, of 2s + 1
#    cells: (S + 1)^2 cells in S + 1 steps.
#  * identical sequences of length n: one cell, one extension of n matches,
#    which a compare of 32 bases at a time covers in floor(n/32) + 1 windows
#    (the last one finds the mismatch or the end).
#  * one substitution at base j of n under (4, 6, 2): score 4 in steps
#    s = 0, 2, 4 (1 + 3 + 5 = 9 cells; s = 2 holds only NULL cells), two
#    extensions (from 0 over j matches, from j + 1 over n - j - 1 matches).
def _counter_failures(align_fn):
    """Counter closed forms that `align_fn(P, T, pen) -> (score, stats)`
    violates (empty list: all hold)."""
    bad = []
    rng = np.random.default_rng(17)
    for n in (0, 1, 5, 31, 32, 33, 63, 64, 65, 100, 200):
        P = bytes(rng.choice(list(b"ACGT"), n).astype(np.uint8))
        sc, st = align_fn(P, P, (4, 6, 2))
        want = dict(cells=1, steps=1, ext_calls=1, ext_windows=n // 32 + 1, ext_matches=n)
        if sc != 0 or any(st[k] != v for k, v in want.items()):
            bad.append(("identical", n, sc, st))
    for n, j in ((100, 50), (100, 0), (100, 99), (64, 31), (64, 32), (200, 131)):
        P = bytearray(rng.choice(list(b"ACGT"), n).astype(np.uint8))
        T = bytearray(P)
        T[j] = b"ACGT"[(b"ACGT".index(T[j]) + 1) % 4]
        sc, st = align_fn(bytes(P), bytes(T), (4, 6, 2))
        want = dict(cells=9, steps=3, ext_calls=2,
                    ext_windows=j // 32 + 1 + (n - j - 1) // 32 + 1, ext_matches=n - 1)
        if sc != 4 or any(st[k] != v for k, v in want.items()):
            bad.append(("substitution", n, j, sc, st))
    pairs = [(bytes(rng.choice(list(b"ACGT"), int(rng.integers(20, 120))).astype(np.uint8)),)
             for _ in range(60)]
    for (P,) in pairs:
        T = bytearray(P)
        for _ in range(int(rng.integers(0, 6))):  # a few random edits
            pos = int(rng.integers(0, max(len(T), 1)))
            kind = int(rng.integers(0, 3))
            if kind == 0 and T:
                T[pos] = b"ACGT"[(b"ACGT".index(T[pos]) + 1) % 4]
            elif kind == 1:
                T[pos:pos] = bytes([b"ACGT"[int(rng.integers(0, 4))]])
            elif T:
                del T[pos]
        T = bytes(T)
        for pen, half in (((4, 6, 2), True), ((1, 0, 1), False)):
            sc, st = align_fn(P, T, pen)
            S = sc // 2 if half else sc
            if S <= min(len(P), len(T)) and (st["cells"] != (S + 1) ** 2 or st["steps"] != S + 1):
                bad.append(("span", pen, len(P), len(T), sc, st))
    return bad


def test_oracle_counters_closed_forms(oracle_lib):
    def fn(P, T, pen):
        sc, _, st = oracle_lib.align(P, T, pen, cigar=False, with_stats=True)
        return sc, st

    assert _counter_failures(fn) == []


# ---- planted mistakes ------------------------------------------------------
# Each mutant changes one line of the oracle's arithmetic the way a plausible
# slip would; the pins must reject every one of them.
MUTANTS = {
    "I_from_k_plus_1": ("int a = wf_get(&t, so, 'M', k - 1);", "int a = wf_get(&t, so, 'M', k + 1);"),
    "no_open_cost": ("int sx = s - x, so = s - o - e, se = s - e;", "int sx = s - x, so = s - e, se = s - e;"),
    "D_extends_from_I": ("int d = wf_get(&t, se, 'D', k + 1);", "int d = wf_get(&t, se, 'I', k + 1);"),
    "extend_skips_first": ("int v = h - k;\n    int run = 0;", "int v = h - k + 1;\n    int run = 0;"),
    "end_row_transposed": ("(v == n && h >= m - te)", "(v == m && h >= m - te)"),
    "end_column_uses_te": ("(h == m && v >= n - pe)", "(h == m && v >= n - te)"),
    "free_start_offset_zero": ("extend(P, n, T, m, k, k > 0 ? k : 0, st)",
                               "extend(P, n, T, m, k, 0 > k ? k : 0, st)"),
    "free_prefix_op_swapped": ("for (int j = 0; j < k; j++) ops[nops++] = OP_I;",
                               "for (int j = 0; j < k; j++) ops[nops++] = OP_D;"),
    "free_suffix_op_swapped": ("for (int j = h - k; j < n; j++) ops[nops++] = OP_D;",
                               "for (int j = h - k; j < n; j++) ops[nops++] = OP_I;"),
    "mismatch_no_advance": ("xx = xx == OFF_NULL ? OFF_NULL : xx + 1;\n            int Mv",
                            "xx = xx == OFF_NULL ? OFF_NULL : xx;\n            int Mv"),
    "backtrace_D_moves_h": ("                k += 1;\n            }\n        }", "                k += 1;\n                h -= 1;\n            }\n        }"),
    # the WF-adaptive reduction
    "adaptive_distance_min": ("return n - v > m - h ? n - v : m - h;", "return n - v < m - h ? n - v : m - h;"),
    "adaptive_distance_sum": ("return n - v > m - h ? n - v : m - h;", "return (n - v) + (m - h);"),
    "adaptive_distance_k_sign": ("    int v = h - k;\n    return n - v", "    int v = h + k;\n    return n - v"),
    "adaptive_width_strict": ("if (w->hi - w->lo + 1 < mwl) return 0;", "if (w->hi - w->lo + 1 <= mwl) return 0;"),
    "adaptive_keep_strict": ("distance_to_end(lo2, w->M[lo2 - w->lo], n, m) > dmin + mdt", "distance_to_end(lo2, w->M[lo2 - w->lo], n, m) >= dmin + mdt"),
    "adaptive_before_extension": (
        "        for (int k = lo; k <= hi; k++) {\n            int i = k - lo;\n            if (w->M[i] != OFF_NULL) w->M[i] = extend(",
        "        if (mwl > 0 && adaptive_reduce(w, n, m, mwl, mdt)) { status = ORACLE_E_NOMEM; goto done; }\n"
        "        for (int k = w->lo; k <= w->hi; k++) {\n            int i = k - w->lo;\n            if (w->M[i] != OFF_NULL) w->M[i] = extend("),
    # counters the benchmark's algorithmic work comes from
    "cells_width_short_by_one": ("st->cells += hi - lo + 1;", "st->cells += hi - lo;"),
    "windows_rounded_up": ("st->ext_windows += run / 32 + 1;", "st->ext_windows += (run + 31) / 32;"),
}


def _build_mutant(tmp_path, name):
    src = open(os.path.join(HERE, "..", "oracle", "wfa_oracle.c")).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, f"mutant {name} no longer applies"
    src = src.replace(old, new, 1)
    d = tmp_path / name
    d.mkdir()
    (d / "wfa_oracle.c").write_text(src)
    hdr = open(os.path.join(HERE, "..", "oracle", "wfa_oracle.h")).read()
    (d / "wfa_oracle.h").write_text(hdr)
    so = d / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", "-pthread", "-o", str(so),
                           str(d / "wfa_oracle.c")])
    return str(so)


def _mutant_caught(so_path) -> bool:
    import ctypes

    lib = ctypes.CDLL(so_path)
    p, i, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    lib.oracle_align.argtypes = [p, i, p, i, i, i, i, i, p, p, i64, p, p]
    lib.oracle_align_ends.argtypes = [p, i, p, i, i, i, i, i, i, i, i, i, p, p, i64, p, p]
    rng = np.random.default_rng(3)
    cases = [(a, b) for a in strings(b"ACG", 3) for b in strings(b"ACG", 3)]
    cases += [(bytes(rng.choice(list(b"ACGT"), 30).astype(np.uint8)),
               bytes(rng.choice(list(b"ACGT"), 27).astype(np.uint8))) for _ in range(20)]
    for pen in [(4, 6, 2), (1, 0, 1)]:
        for P, T in cases:
            n, m = len(P), len(T)
            runs = (ctypes.c_uint32 * (n + m + 1))()
            sc = ctypes.c_int32()
            nr = ctypes.c_int64()
            # run the mutant in a child-safe way: bound the work by a step cap
            rc = lib.oracle_align(ctypes.create_string_buffer(P, n + 1), n,
                                  ctypes.create_string_buffer(T, m + 1), m, *pen, 1,
                                  ctypes.byref(sc), runs, n + m + 1, ctypes.byref(nr), None)
            if rc != 0 or sc.value != brute.gotoh(P, T, *pen)[0]:
                return True
            try:
                if brute.check_cigar(P, T, list(runs)[:nr.value], *pen) != sc.value:
                    return True
            except AssertionError:
                return True
    # the work counters
    class _St(ctypes.Structure):
        _fields_ = [(f, ctypes.c_int64) for f in
                    ("cells", "steps", "ext_calls", "ext_windows", "ext_matches")]

    def counted(P, T, pen):
        n, m = len(P), len(T)
        st = _St()
        sc = ctypes.c_int32()
        nr = ctypes.c_int64()
        rc = lib.oracle_align(ctypes.create_string_buffer(P, n + 1), n,
                              ctypes.create_string_buffer(T, m + 1), m, *pen, 0,
                              ctypes.byref(sc), None, 0, ctypes.byref(nr), ctypes.byref(st))
        if rc != 0:
            raise RuntimeError("oracle_align failed")
        return sc.value, {f: int(getattr(st, f)) for f, _ in st._fields_}

    try:
        if _counter_failures(counted):
            return True
    except RuntimeError:
        return True
    # the WF-adaptive heuristic
    lib.oracle_align_adaptive.argtypes = [p, i, p, i, i, i, i, i, i, i, p, p, i64, p, p]

    def adaptive(P, T, pen, ad):
        n, m = len(P), len(T)
        runs = (ctypes.c_uint32 * (n + m + 1))()
        sc = ctypes.c_int32()
        nr = ctypes.c_int64()
        rc = lib.oracle_align_adaptive(ctypes.create_string_buffer(P, n + 1), n,
                                       ctypes.create_string_buffer(T, m + 1), m, *pen, *ad, 1,
                                       ctypes.byref(sc), runs, n + m + 1, ctypes.byref(nr), None)
        if rc != 0:
            raise AssertionError("oracle_align_adaptive failed")
        return sc.value, list(runs)[:nr.value]

    try:
        for P, T, ad, score, cigar in ADAPTIVE_WORKED:
            s, runs = adaptive(P, T, (4, 6, 2), ad)
            if s != score or "".join(f"{r >> 4}{'MXID'[r & 15]}" for r in runs) != cigar:
                return True
        for P, T in cases[::5]:
            s, runs = adaptive(P, T, (4, 6, 2), (1, max(len(P), len(T))))
            if s != brute.gotoh(P, T, 4, 6, 2)[0]:
                return True
            for ad in [(1, 0), (3, 1)]:
                s, runs = adaptive(P, T, (4, 6, 2), ad)
                c = brute.check_cigar(P, T, runs, 4, 6, 2)
                if s < brute.gotoh(P, T, 4, 6, 2)[0] or c > s or c < brute.gotoh(P, T, 4, 6, 2)[0]:
                    return True
    except AssertionError:
        return True
    # ends-free cases
    for pen in [(4, 6, 2), (1, 0, 1)]:
        for ends in ENDS_SHORT:
            for P, T in cases[:200:3] + cases[-6:]:
                n, m = len(P), len(T)
                runs = (ctypes.c_uint32 * (n + m + 1))()
                sc = ctypes.c_int32()
                nr = ctypes.c_int64()
                rc = lib.oracle_align_ends(ctypes.create_string_buffer(P, n + 1), n,
                                           ctypes.create_string_buffer(T, m + 1), m, *pen, *ends,
                                           1, ctypes.byref(sc), runs, n + m + 1, ctypes.byref(nr),
                                           None)
                if rc != 0 or sc.value != brute.gotoh_ends(P, T, *pen, ends):
                    return True
                try:
                    if brute.check_cigar_ends(P, T, list(runs)[:nr.value], *pen, ends) != sc.value:
                        return True
                except AssertionError:
                    return True
    return False


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    so = _build_mutant(tmp_path, name)
    # mutants can loop forever (never reaching the end cell): run in a child
    import multiprocessing as mp

    ctx = mp.get_context("fork")
    q = ctx.Queue()
    def child():
        import faulthandler

        faulthandler.disable()  # a mutant that crashes is caught; no traceback dump
        q.put(_mutant_caught(so))

    proc = ctx.Process(target=child)
    proc.start()
    proc.join(5)
    if proc.is_alive():
        proc.kill()
        proc.join()
        return  # non-termination is itself a caught mistake
    if proc.exitcode != 0:
        return  # crash: caught
    assert q.get(timeout=5), f"mutant {name} passed the pins"
