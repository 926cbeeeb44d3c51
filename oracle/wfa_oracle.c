/*
 * CPU oracle for batched gap-affine global alignment with the wavefront
 * algorithm (WFA).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP library is checked against.  It shares no code,
 * header, table or helper with the library; only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg load it.
 *
 * What is computed.  The paper (Introduction and Methods) aligns read pairs
 * with WFA, the gap-affine wavefront algorithm of Marco-Sola, Moure, Moreto
 * and Espinosa (Bioinformatics 37(4), 2021; "WFA" below), and writes one
 * result per pair.  WFA returns the optimal gap-affine score
 *
 *   score(P, T) = min over global alignments of
 *                 x * #mismatches + sum over maximal gap runs (o + e * len)
 *
 * and one optimal alignment.  Here P (length n) is the pattern, T (length m)
 * the text, x the mismatch penalty, o the gap-open and e the gap-extend
 * penalty; matches cost 0.
 *
 * Steps, in WFA's order and notation:
 *   - diagonal k = h - v, offset = h (position in T); cell (v, h) means
 *     P[0..v) is aligned with T[0..h)                       (WFA, definitions)
 *   - wavefront components M_s, I_s, D_s map a diagonal to its furthest
 *     reaching offset with score s, or to nothing (NULL)     (WFA, definitions)
 *   - s = 0: M_0[0] = 0, then extend                         (WFA, initial condition)
 *   - for s > 0:                                             (WFA, recurrences)
 *       I_s[k] = max{ M_{s-o-e}[k-1] + 1, I_{s-e}[k-1] + 1 }
 *       D_s[k] = max{ M_{s-o-e}[k+1],     D_{s-e}[k+1] }
 *       M_s[k] = max{ M_{s-x}[k] + 1, I_s[k], D_s[k] }
 *     then extend every M_s[k] along matching characters    (WFA, extend)
 *   - the alignment ends at the first s with M_s[m-n] == m   (WFA, termination)
 *   - the alignment is read back from the kept wavefronts    (WFA, backtrace)
 *
 * Ends-free variant (global alignment is the case of four zeros).  With
 * pattern_begin_free pb, pattern_end_free pe, text_begin_free tb and
 * text_end_free te (each clipped to the sequence's length), an alignment
 * may leave unaligned at no cost a prefix of at most pb pattern bases or
 * one of at most tb text bases, and a suffix of at most pe pattern bases or
 * one of at most te text bases:
 *
 *   score = min over the allowed (start, end) of the global score of
 *           P[vb..ve) against T[hb..he), where (vb, hb) is (v, 0) with
 *           v <= pb or (0, h) with h <= tb, and (ve, he) is (v, m) with
 *           v >= n - pe or (n, h) with h >= m - te.
 *
 * In wavefront terms: s = 0 holds M_0[k] = max(k, 0) for k in [-pb, tb]
 * (each extended); the alignment ends at the first s holding an M cell on
 * the last text column with v >= n - pe or on the last pattern row with
 * h >= m - te.  Readings: of several such cells the one on the lowest
 * diagonal ends the alignment; the CIGAR spells both sequences whole, the
 * free prefix and suffix as I (text) or D (pattern) runs that cost nothing
 * (a free run and an adjacent paid gap of the same op share one run).
 *
 * Readings where WFA leaves a choice (each is listed with its reason in the
 * design notes of the repository):
 *   - a candidate offset c on diagonal k is admissible only if it is a real
 *     cell: c <= m and c - k <= n.  Inadmissible candidates are dropped
 *     before the maximum is taken (never "max, then drop").
 *   - a wavefront at score s spans [lo, hi] with lo one below and hi one
 *     above the extreme diagonals of its source wavefronts, clipped to
 *     [-n, m]; a score with no source wavefront has no wavefront.
 *   - backtrace tie-break: in M, mismatch (same diagonal) before I (from
 *     k-1) before D (from k+1); in I and D, gap-open (from M) before
 *     gap-extend.
 *   - CIGAR ops: M = match only, X = mismatch, I consumes one text base,
 *     D consumes one pattern base; runs are stored as len << 4 | op with
 *     op codes M=0, X=1, I=2, D=3.
 *   - score-only mode keeps only the wavefronts still reachable by the
 *     recurrences (scores s - max(x, o+e) and later).
 *
 * The oracle accepts any byte values; characters compare as raw bytes.
 *
 * Pins (tests/test_oracle_pins.py): scores against exhaustive enumeration and
 * the textbook Gotoh DP, the Levenshtein special case and closed forms;
 * CIGARs against Gotoh's traceback wherever the optimal alignment is unique,
 * and against spelling / re-scoring invariants everywhere.  Which of several
 * optimal alignments is reported follows only the tie-break reading above:
 * for pairs with more than one optimum the CIGAR choice is "parity unpinned"
 * (fixed by this oracle, with no outside reference).
 */
#include <limits.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "wfa_oracle.h"

#define OFF_NULL (INT_MIN / 2)

typedef struct {
    int present;
    int lo, hi;
    int *M, *I, *D; /* indexed by k - lo */
} wavefront;

typedef struct {
    wavefront *wf;
    int cap;
} wf_table;

static int wf_get(const wf_table *t, int s, char comp, int k) {
    if (s < 0 || s >= t->cap) return OFF_NULL;
    const wavefront *w = &t->wf[s];
    if (!w->present || k < w->lo || k > w->hi) return OFF_NULL;
    int i = k - w->lo;
    return comp == 'M' ? w->M[i] : comp == 'I' ? w->I[i] : w->D[i];
}

static int wf_present(const wf_table *t, int s) {
    return s >= 0 && s < t->cap && t->wf[s].present;
}

static int admissible(int c, int k, int n, int m) {
    if (c == OFF_NULL || c < 0) return 0;
    int lim = m < n + k ? m : n + k;
    return c <= lim;
}

static int max_or_null(int a, int b) {
    if (a == OFF_NULL) return b;
    if (b == OFF_NULL) return a;
    return a > b ? a : b;
}

static int grow(wf_table *t, int s) {
    if (s < t->cap) return 0;
    int ncap = t->cap ? t->cap : 64;
    while (ncap <= s) ncap *= 2;
    wavefront *nw = (wavefront *)realloc(t->wf, sizeof(wavefront) * (size_t)ncap);
    if (!nw) return -1;
    memset(nw + t->cap, 0, sizeof(wavefront) * (size_t)(ncap - t->cap));
    t->wf = nw;
    t->cap = ncap;
    return 0;
}

static void wf_free(wavefront *w) {
    free(w->M);
    free(w->I);
    free(w->D);
    w->M = w->I = w->D = NULL;
    w->present = 0;
}

static int wf_alloc(wavefront *w, int lo, int hi) {
    int len = hi - lo + 1;
    w->lo = lo;
    w->hi = hi;
    w->M = (int *)malloc(sizeof(int) * (size_t)len);
    w->I = (int *)malloc(sizeof(int) * (size_t)len);
    w->D = (int *)malloc(sizeof(int) * (size_t)len);
    if (!w->M || !w->I || !w->D) return -1;
    for (int i = 0; i < len; i++) w->M[i] = w->I[i] = w->D[i] = OFF_NULL;
    w->present = 1;
    return 0;
}

/* Extend along matching characters (WFA, extend step). */
static int extend(const uint8_t *P, int n, const uint8_t *T, int m, int k, int h,
                  oracle_stats *st) {
    int v = h - k;
    int run = 0;
    while (v < n && h < m && P[v] == T[h]) {
        v++;
        h++;
        run++;
    }
    if (st) {
        st->ext_calls++;
        st->ext_matches += run;
        st->ext_windows += run / 32 + 1;
    }
    return h;
}

enum { OP_M = 0, OP_X = 1, OP_I = 2, OP_D = 3 };

/* Whether the M cell at offset h on diagonal k may end an ends-free
 * alignment: on the last text column with at most pe pattern bases left, or
 * on the last pattern row with at most te text bases left. */
static int is_end_cell(int k, int h, int n, int m, int pe, int te) {
    int v = h - k;
    return (h == m && v >= n - pe) || (v == n && h >= m - te);
}

/* Lowest diagonal of wavefront w whose M cell ends the alignment, or
 * INT_MIN if none does. */
static int end_diagonal(const wavefront *w, int n, int m, int pe, int te) {
    for (int k = w->lo; k <= w->hi; k++) {
        int h = w->M[k - w->lo];
        if (h != OFF_NULL && is_end_cell(k, h, n, m, pe, te)) return k;
    }
    return INT_MIN;
}

static int clip(int v, int hi) { return v < hi ? v : hi; }

/* Distance from the furthest point of diagonal k (offset h) to the end cell:
 * the larger of the pattern and the text bases still to cover. */
static int distance_to_end(int k, int h, int n, int m) {
    int v = h - k;
    return n - v > m - h ? n - v : m - h;
}

/* WF-adaptive reduction, the heuristic mode of the WFA paper that the
 * method builds on (cited in section 1, Introduction and Methods): once
 * a wavefront holds at least mwl diagonals, the distance of each diagonal's
 * furthest point (v, h) to the end cell (n, m) is the larger of the pattern
 * and the text bases it still has to cover, max(n - v, m - h); the diagonals
 * at either end of the wavefront whose distance exceeds the smallest
 * distance by more than mdt (or that hold no offset) are dropped, and the
 * wavefront keeps the range between the outermost diagonals it keeps.
 * Returns -1 when out of memory.  Readings: the width counts every diagonal
 * of the wavefront's span, those without an offset included; a wavefront
 * without any offset is left as it is; the reduction applies after the
 * extension and the end test of the step, and not to a step that ends the
 * alignment; the score is the step that reaches the end, whose path may
 * close a gap and open another of the same kind at once (the CIGAR merges
 * them into one run, one opening cheaper than the score). */
static int adaptive_reduce(wavefront *w, int n, int m, int mwl, int mdt) {
    if (w->hi - w->lo + 1 < mwl) return 0;
    int dmin = INT_MAX;
    for (int k = w->lo; k <= w->hi; k++) {
        int h = w->M[k - w->lo];
        if (h != OFF_NULL && distance_to_end(k, h, n, m) < dmin) dmin = distance_to_end(k, h, n, m);
    }
    if (dmin == INT_MAX) return 0;
    /* the kept range: from the outermost diagonals within dmin + mdt */
    int lo2 = w->lo, hi2 = w->hi;
    while (w->M[lo2 - w->lo] == OFF_NULL || distance_to_end(lo2, w->M[lo2 - w->lo], n, m) > dmin + mdt)
        lo2++;
    while (w->M[hi2 - w->lo] == OFF_NULL || distance_to_end(hi2, w->M[hi2 - w->lo], n, m) > dmin + mdt)
        hi2--;
    if (lo2 == w->lo && hi2 == w->hi) return 0;
    wavefront nw = {0, 0, 0, NULL, NULL, NULL};
    if (wf_alloc(&nw, lo2, hi2)) { wf_free(&nw); return -1; }
    for (int k = lo2; k <= hi2; k++) {
        nw.M[k - lo2] = w->M[k - w->lo];
        nw.I[k - lo2] = w->I[k - w->lo];
        nw.D[k - lo2] = w->D[k - w->lo];
    }
    wf_free(w);
    *w = nw;
    return 0;
}

int oracle_align(const uint8_t *P, int n, const uint8_t *T, int m,
                 int x, int o, int e, int want_cigar,
                 int32_t *score_out, uint32_t *runs, int64_t runs_cap, int64_t *nruns_out,
                 oracle_stats *st) {
    return oracle_align_ends(P, n, T, m, x, o, e, 0, 0, 0, 0, want_cigar, score_out, runs,
                             runs_cap, nruns_out, st);
}

/* The steps shared by every entry point: ends-free bounds (all zero for
 * global alignment) and the WF-adaptive parameters (mwl = 0: exact). */
static int align_core(const uint8_t *P, int n, const uint8_t *T, int m,
                      int x, int o, int e, int pb, int pe, int tb, int te, int mwl, int mdt,
                      int want_cigar, int32_t *score_out, uint32_t *runs, int64_t runs_cap,
                      int64_t *nruns_out, oracle_stats *st);

int oracle_align_ends(const uint8_t *P, int n, const uint8_t *T, int m,
                      int x, int o, int e, int pb, int pe, int tb, int te, int want_cigar,
                      int32_t *score_out, uint32_t *runs, int64_t runs_cap, int64_t *nruns_out,
                      oracle_stats *st) {
    return align_core(P, n, T, m, x, o, e, pb, pe, tb, te, 0, 0, want_cigar, score_out, runs,
                      runs_cap, nruns_out, st);
}

int oracle_align_adaptive(const uint8_t *P, int n, const uint8_t *T, int m, int x, int o, int e,
                          int min_wavefront_length, int max_distance_threshold, int want_cigar,
                          int32_t *score_out, uint32_t *runs, int64_t runs_cap, int64_t *nruns_out,
                          oracle_stats *st) {
    if (min_wavefront_length < 0 || max_distance_threshold < 0) return ORACLE_E_INVAL;
    return align_core(P, n, T, m, x, o, e, 0, 0, 0, 0, min_wavefront_length,
                      max_distance_threshold, want_cigar, score_out, runs, runs_cap, nruns_out, st);
}

static int align_core(const uint8_t *P, int n, const uint8_t *T, int m,
                      int x, int o, int e, int pb, int pe, int tb, int te, int mwl, int mdt,
                      int want_cigar, int32_t *score_out, uint32_t *runs, int64_t runs_cap,
                      int64_t *nruns_out, oracle_stats *st) {
    if (x <= 0 || e <= 0 || o < 0 || n < 0 || m < 0) return ORACLE_E_INVAL;
    if (pb < 0 || pe < 0 || tb < 0 || te < 0) return ORACLE_E_INVAL;
    pb = clip(pb, n);
    pe = clip(pe, n);
    tb = clip(tb, m);
    te = clip(te, m);
    wf_table t = {NULL, 0};
    int status = ORACLE_OK;
    int keep = x > o + e ? x : o + e; /* score-only mode: how far back sources reach */
    int S = -1, end_k = INT_MIN;

    /* s = 0: the free starts, each extended */
    if (grow(&t, 0) || wf_alloc(&t.wf[0], -pb, tb)) { status = ORACLE_E_NOMEM; goto done; }
    for (int k = -pb; k <= tb; k++)
        t.wf[0].M[k + pb] = extend(P, n, T, m, k, k > 0 ? k : 0, st);
    if (st) { st->cells += pb + tb + 1; st->steps += 1; }
    end_k = end_diagonal(&t.wf[0], n, m, pe, te);
    if (end_k != INT_MIN) S = 0;
    if (S < 0 && mwl > 0 && adaptive_reduce(&t.wf[0], n, m, mwl, mdt)) { status = ORACLE_E_NOMEM; goto done; }

    for (int s = 1; S < 0; s++) {
        if (grow(&t, s)) { status = ORACLE_E_NOMEM; goto done; }
        int sx = s - x, so = s - o - e, se = s - e;
        int lo = INT_MAX, hi = INT_MIN;
        if (wf_present(&t, sx)) { lo = t.wf[sx].lo < lo ? t.wf[sx].lo : lo; hi = t.wf[sx].hi > hi ? t.wf[sx].hi : hi; }
        if (wf_present(&t, so)) { lo = t.wf[so].lo < lo ? t.wf[so].lo : lo; hi = t.wf[so].hi > hi ? t.wf[so].hi : hi; }
        if (wf_present(&t, se)) { lo = t.wf[se].lo < lo ? t.wf[se].lo : lo; hi = t.wf[se].hi > hi ? t.wf[se].hi : hi; }
        if (lo == INT_MAX) continue; /* no source wavefront: no wavefront at s */
        lo -= 1;
        hi += 1;
        if (lo < -n) lo = -n;
        if (hi > m) hi = m;
        wavefront *w = &t.wf[s];
        if (wf_alloc(w, lo, hi)) { status = ORACLE_E_NOMEM; goto done; }
        if (st) { st->cells += hi - lo + 1; st->steps += 1; }
        for (int k = lo; k <= hi; k++) {
            int i = k - lo;
            /* I: gap consuming a text base, entered from diagonal k-1 */
            int a = wf_get(&t, so, 'M', k - 1);
            int b = wf_get(&t, se, 'I', k - 1);
            a = a == OFF_NULL ? OFF_NULL : a + 1;
            b = b == OFF_NULL ? OFF_NULL : b + 1;
            int Iv = max_or_null(admissible(a, k, n, m) ? a : OFF_NULL,
                                 admissible(b, k, n, m) ? b : OFF_NULL);
            /* D: gap consuming a pattern base, entered from diagonal k+1 */
            int c = wf_get(&t, so, 'M', k + 1);
            int d = wf_get(&t, se, 'D', k + 1);
            int Dv = max_or_null(admissible(c, k, n, m) ? c : OFF_NULL,
                                 admissible(d, k, n, m) ? d : OFF_NULL);
            /* M: mismatch along diagonal k, or the end of a gap */
            int xx = wf_get(&t, sx, 'M', k);
            xx = xx == OFF_NULL ? OFF_NULL : xx + 1;
            int Mv = max_or_null(admissible(xx, k, n, m) ? xx : OFF_NULL,
                                 max_or_null(Iv, Dv));
            w->I[i] = Iv;
            w->D[i] = Dv;
            w->M[i] = Mv;
        }
        for (int k = lo; k <= hi; k++) {
            int i = k - lo;
            if (w->M[i] != OFF_NULL) w->M[i] = extend(P, n, T, m, k, w->M[i], st);
        }
        end_k = end_diagonal(w, n, m, pe, te);
        if (end_k != INT_MIN) S = s;
        if (S < 0 && mwl > 0 && adaptive_reduce(w, n, m, mwl, mdt)) { status = ORACLE_E_NOMEM; goto done; }
        if (!want_cigar && s - keep - 1 >= 0 && s - keep - 1 < t.cap) wf_free(&t.wf[s - keep - 1]);
    }
    *score_out = S;

    if (want_cigar) {
        /* backtrace from the end cell, ops collected in reverse */
        int64_t cap = (int64_t)n + m + 1;
        uint8_t *ops = (uint8_t *)malloc((size_t)cap);
        int64_t nops = 0;
        if (!ops) { status = ORACLE_E_NOMEM; goto done; }
        int s = S, k = end_k, h = wf_get(&t, S, 'M', end_k);
        /* the free suffix (ops are collected last to first) */
        for (int j = h - k; j < n; j++) ops[nops++] = OP_D;
        for (int j = h; j < m; j++) ops[nops++] = OP_I;
        char comp = 'M';
        for (;;) {
            if (comp == 'M') {
                int h0;
                int xx = OFF_NULL, Iv = OFF_NULL, Dv = OFF_NULL;
                if (s == 0) {
                    h0 = k > 0 ? k : 0; /* M_0[k] before extension */
                } else {
                    xx = wf_get(&t, s - x, 'M', k);
                    xx = xx == OFF_NULL ? OFF_NULL : xx + 1;
                    if (!admissible(xx, k, n, m)) xx = OFF_NULL;
                    Iv = wf_get(&t, s, 'I', k);
                    Dv = wf_get(&t, s, 'D', k);
                    h0 = max_or_null(xx, max_or_null(Iv, Dv));
                }
                for (int j = 0; j < h - h0; j++) ops[nops++] = OP_M;
                h = h0;
                if (s == 0) {
                    /* the free prefix */
                    for (int j = 0; j < k; j++) ops[nops++] = OP_I;
                    for (int j = 0; j < -k; j++) ops[nops++] = OP_D;
                    break;
                }
                if (xx != OFF_NULL && xx == h0) {
                    ops[nops++] = OP_X;
                    s -= x;
                    h -= 1;
                } else if (Iv != OFF_NULL && Iv == h0) {
                    comp = 'I';
                } else {
                    comp = 'D';
                }
            } else if (comp == 'I') {
                ops[nops++] = OP_I;
                int a = wf_get(&t, s - o - e, 'M', k - 1);
                a = a == OFF_NULL ? OFF_NULL : a + 1;
                if (admissible(a, k, n, m) && a == h) {
                    s -= o + e;
                    comp = 'M';
                } else {
                    s -= e;
                }
                k -= 1;
                h -= 1;
            } else {
                ops[nops++] = OP_D;
                int c = wf_get(&t, s - o - e, 'M', k + 1);
                if (admissible(c, k, n, m) && c == h) {
                    s -= o + e;
                    comp = 'M';
                } else {
                    s -= e;
                }
                k += 1;
            }
        }
        /* reverse into alignment order and run-length encode */
        int64_t nr = 0;
        int64_t i = nops - 1;
        while (i >= 0) {
            uint8_t op = ops[i];
            int64_t len = 0;
            while (i >= 0 && ops[i] == op) { len++; i--; }
            if (nr < runs_cap) runs[nr] = (uint32_t)(len << 4 | op);
            nr++;
        }
        free(ops);
        *nruns_out = nr;
        if (nr > runs_cap) status = ORACLE_E_CAPACITY;
    } else if (nruns_out) {
        *nruns_out = 0;
    }

done:
    for (int s = 0; s < t.cap; s++) wf_free(&t.wf[s]);
    free(t.wf);
    return status;
}

/* ---- batch driver: static chunks over a pthread pool -------------------- */

typedef struct {
    const uint8_t *pbuf, *tbuf;
    const uint64_t *poff, *toff;
    const uint32_t *plen, *tlen;
    int x, o, e, want_cigar;
    int pb, pe, tb, te;
    int mwl, mdt;
    int32_t *scores;
    uint32_t *runs;    /* slot-strided: pair i writes runs[i * slot ...] */
    int64_t slot;
    int64_t *nruns;
    int32_t *status;
    int64_t begin, end;
    oracle_stats st;
} job_t;

static void *run_job(void *arg) {
    job_t *j = (job_t *)arg;
    for (int64_t i = j->begin; i < j->end; i++) {
        int64_t nr = 0;
        int rc = align_core(j->pbuf + j->poff[i], (int)j->plen[i], j->tbuf + j->toff[i],
                            (int)j->tlen[i], j->x, j->o, j->e, j->pb, j->pe, j->tb, j->te, j->mwl,
                            j->mdt, j->want_cigar, &j->scores[i],
                            j->runs ? j->runs + i * j->slot : NULL, j->slot, &nr, &j->st);
        if (j->nruns) j->nruns[i] = nr;
        if (j->status) j->status[i] = rc;
    }
    return NULL;
}

int oracle_align_batch(const uint8_t *pbuf, const uint64_t *poff, const uint32_t *plen,
                       const uint8_t *tbuf, const uint64_t *toff, const uint32_t *tlen,
                       int64_t count, int x, int o, int e, int want_cigar,
                       int32_t *scores, uint32_t *runs, int64_t slot, int64_t *nruns,
                       int32_t *status, int threads, oracle_stats *st) {
    return oracle_align_batch_ends(pbuf, poff, plen, tbuf, toff, tlen, count, x, o, e, 0, 0, 0,
                                   0, want_cigar, scores, runs, slot, nruns, status, threads, st);
}

static int batch_core(const uint8_t *pbuf, const uint64_t *poff, const uint32_t *plen,
                      const uint8_t *tbuf, const uint64_t *toff, const uint32_t *tlen,
                      int64_t count, int x, int o, int e, int pb, int pe, int tb, int te,
                      int mwl, int mdt, int want_cigar, int32_t *scores, uint32_t *runs,
                      int64_t slot, int64_t *nruns, int32_t *status, int threads,
                      oracle_stats *st);

int oracle_align_batch_ends(const uint8_t *pbuf, const uint64_t *poff, const uint32_t *plen,
                            const uint8_t *tbuf, const uint64_t *toff, const uint32_t *tlen,
                            int64_t count, int x, int o, int e, int pb, int pe, int tb, int te,
                            int want_cigar, int32_t *scores, uint32_t *runs, int64_t slot,
                            int64_t *nruns, int32_t *status, int threads, oracle_stats *st) {
    return batch_core(pbuf, poff, plen, tbuf, toff, tlen, count, x, o, e, pb, pe, tb, te, 0, 0,
                      want_cigar, scores, runs, slot, nruns, status, threads, st);
}

int oracle_align_batch_adaptive(const uint8_t *pbuf, const uint64_t *poff, const uint32_t *plen,
                                const uint8_t *tbuf, const uint64_t *toff, const uint32_t *tlen,
                                int64_t count, int x, int o, int e, int min_wavefront_length,
                                int max_distance_threshold, int want_cigar, int32_t *scores,
                                uint32_t *runs, int64_t slot, int64_t *nruns, int32_t *status,
                                int threads, oracle_stats *st) {
    if (min_wavefront_length < 0 || max_distance_threshold < 0) return ORACLE_E_INVAL;
    return batch_core(pbuf, poff, plen, tbuf, toff, tlen, count, x, o, e, 0, 0, 0, 0,
                      min_wavefront_length, max_distance_threshold, want_cigar, scores, runs, slot,
                      nruns, status, threads, st);
}

static int batch_core(const uint8_t *pbuf, const uint64_t *poff, const uint32_t *plen,
                      const uint8_t *tbuf, const uint64_t *toff, const uint32_t *tlen,
                      int64_t count, int x, int o, int e, int pb, int pe, int tb, int te,
                      int mwl, int mdt, int want_cigar, int32_t *scores, uint32_t *runs,
                      int64_t slot, int64_t *nruns, int32_t *status, int threads,
                      oracle_stats *st) {
    if (threads < 1) threads = 1;
    if (threads > 1024) threads = 1024;
    job_t *jobs = (job_t *)calloc((size_t)threads, sizeof(job_t));
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    if (!jobs || !tid) { free(jobs); free(tid); return ORACLE_E_NOMEM; }
    for (int t = 0; t < threads; t++) {
        job_t *j = &jobs[t];
        j->pbuf = pbuf; j->tbuf = tbuf; j->poff = poff; j->toff = toff;
        j->plen = plen; j->tlen = tlen; j->x = x; j->o = o; j->e = e;
        j->pb = pb; j->pe = pe; j->tb = tb; j->te = te;
        j->mwl = mwl; j->mdt = mdt;
        j->want_cigar = want_cigar; j->scores = scores; j->runs = runs; j->slot = slot;
        j->nruns = nruns; j->status = status;
        j->begin = count * t / threads;
        j->end = count * (t + 1) / threads;
    }
    int started = 0;
    for (int t = 1; t < threads; t++)
        if (pthread_create(&tid[t], NULL, run_job, &jobs[t]) == 0) started = t; else break;
    run_job(&jobs[0]);
    for (int t = 1; t <= started; t++) pthread_join(tid[t], NULL);
    for (int t = started + 1; t < threads; t++) run_job(&jobs[t]); /* threads that failed to start */
    if (st) {
        memset(st, 0, sizeof(*st));
        for (int t = 0; t < threads; t++) {
            st->cells += jobs[t].st.cells;
            st->steps += jobs[t].st.steps;
            st->ext_calls += jobs[t].st.ext_calls;
            st->ext_windows += jobs[t].st.ext_windows;
            st->ext_matches += jobs[t].st.ext_matches;
        }
    }
    free(jobs);
    free(tid);
    return ORACLE_OK;
}

/* ---- 2-bit encoding of the library's packed input format ----------------
 * Plain definition: base i of a sequence occupies bits 2*(i mod 32) and
 * 2*(i mod 32)+1 of 64-bit word i / 32 (least significant pair first), with
 * A=0, C=1, G=2, T=3, upper or lower case.  Words past the sequence are 0.
 * Returns the index of the first byte outside ACGTacgt, or -1.            */
int64_t oracle_pack2bit(const uint8_t *seq, int64_t len, uint64_t *words, int64_t nwords) {
    for (int64_t w = 0; w < nwords; w++) words[w] = 0;
    for (int64_t i = 0; i < len; i++) {
        uint64_t code;
        switch (seq[i]) {
        case 'A': case 'a': code = 0; break;
        case 'C': case 'c': code = 1; break;
        case 'G': case 'g': code = 2; break;
        case 'T': case 't': code = 3; break;
        default: return i;
        }
        words[i / 32] |= code << (2 * (i % 32));
    }
    return -1;
}
