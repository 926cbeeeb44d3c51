/*
 * Seeded synthetic read-pair generator.
 *
 * This module only produces input bytes.  It contains none of the alignment
 * arithmetic: both the CPU oracle and the HIP library consume what it writes.
 *
 * Every pair is generated from its own counter-derived random stream, so any
 * sub-range of a batch can be produced independently and in parallel, and the
 * bytes of pair i never depend on how many pairs are generated around it.
 *
 * Random source: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), the 64-bit mixer with the
 * golden-ratio increment.  The per-pair stream starts from
 *   state0 = mix64(seed ^ mix64(pair_index + 1)).
 *
 * Read model (shapes of the paper's workload: pairs of 100 bp reads whose
 * texts differ from the patterns by a given fraction of edits, Results):
 *   - pattern: i.i.d. uniform over A, C, G, T;
 *   - the number of edit events is fixed, or round(r * n) with r drawn per pair;
 *   - event positions are distinct, drawn uniformly from [0, n) (Floyd's
 *     sampling), and processed in ascending order;
 *   - each event is a substitution, an insertion or a deletion with
 *     probability 1/3 each; a substitution picks one of the three other
 *     bases, an insertion places uniform bases before the position, a
 *     deletion removes the base at the position;
 *   - in run mode, insertion/deletion lengths are geometric(1/2) on {1,2,...}
 *     truncated at 64, and a deletion run stops at the next event position.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#include "synth.h"

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

typedef struct { uint64_t s; } rng_t;

static inline uint64_t rng_next(rng_t *r) {
    r->s += 0x9E3779B97F4A7C15ULL;
    return mix64(r->s);
}

/* uniform integer in [0, k) by the multiply-high method (k >= 1) */
static inline uint32_t rng_below(rng_t *r, uint32_t k) {
    return (uint32_t)(((unsigned __int128)rng_next(r) * k) >> 64);
}

/* uniform double in [0, 1) with 53 random bits */
static inline double rng_unit(rng_t *r) {
    return (double)(rng_next(r) >> 11) * (1.0 / 9007199254740992.0);
}

static const char BASES[4] = {'A', 'C', 'G', 'T'};

static inline int base_index(uint8_t b) {
    switch (b) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    default: return 3;
    }
}

static uint32_t draw_length(const synth_spec *sp, rng_t *r) {
    switch (sp->len_dist) {
    case SYNTH_LEN_FIXED:
        return sp->n_lo;
    case SYNTH_LEN_UNIFORM:
        return sp->n_lo + rng_below(r, sp->n_hi - sp->n_lo + 1);
    default: { /* log-uniform on [n_lo, n_hi], rounded */
        double a = log((double)sp->n_lo), b = log((double)sp->n_hi);
        double n = floor(exp(a + (b - a) * rng_unit(r)) + 0.5);
        if (n < sp->n_lo) n = sp->n_lo;
        if (n > sp->n_hi) n = sp->n_hi;
        return (uint32_t)n;
    }
    }
}

static uint32_t draw_events(const synth_spec *sp, rng_t *r, uint32_t n) {
    uint32_t k;
    if (sp->edit_mode == SYNTH_EDITS_FIXED) {
        k = sp->edits;
    } else {
        double rate = sp->r_lo + (sp->r_hi - sp->r_lo) * rng_unit(r);
        k = (uint32_t)floor(rate * (double)n + 0.5);
    }
    return k > n ? n : k;
}

static uint32_t draw_run(const synth_spec *sp, rng_t *r) {
    if (!sp->runs) return 1;
    uint32_t len = 1;
    while (len < 64 && (rng_next(r) >> 63)) len++;
    return len;
}

/*
 * Generate pair `idx`.  If pat/txt are NULL only the lengths are produced;
 * the random draws are identical either way.  `mark` is a caller scratch
 * bitmap of at least (n_hi/64 + 1) words.
 */
static void gen_pair(const synth_spec *sp, uint64_t seed, uint64_t idx,
                     uint8_t *pat, uint8_t *txt, uint32_t *pn, uint32_t *tm,
                     uint64_t *mark) {
    rng_t r;
    r.s = mix64(seed ^ mix64(idx + 1));

    uint32_t n = draw_length(sp, &r);
    uint32_t k = draw_events(sp, &r, n);

    /* pattern bases are always drawn so the event stream is independent of
     * whether the caller wants bytes */
    for (uint32_t i = 0; i < n; i++) {
        uint8_t b = (uint8_t)BASES[rng_next(&r) >> 62];
        if (pat) pat[i] = b;
    }

    /* Floyd's algorithm: k distinct positions of [0, n) */
    uint32_t words = n / 64 + 1;
    memset(mark, 0, words * sizeof(uint64_t));
    for (uint32_t j = n - k; j < n; j++) {
        uint32_t t = rng_below(&r, j + 1);
        if (mark[t >> 6] >> (t & 63) & 1) t = j;
        mark[t >> 6] |= 1ULL << (t & 63);
    }

    /* walk the pattern left to right and apply events at marked positions */
    uint32_t out = 0;
    uint32_t skip_until = 0; /* deletion run in progress covers [p, skip_until) */
    for (uint32_t p = 0; p < n; p++) {
        int marked = (int)(mark[p >> 6] >> (p & 63) & 1);
        if (!marked && p < skip_until) continue;
        /* a new event position ends any deletion run */
        skip_until = 0;
        if (!marked) {
            if (txt) txt[out] = pat ? pat[p] : 0;
            out++;
            continue;
        }
        uint32_t type = rng_below(&r, 3);
        if (type == 0) { /* substitution */
            uint32_t d = 1 + rng_below(&r, 3);
            if (txt) txt[out] = (uint8_t)BASES[(base_index(pat ? pat[p] : 'A') + d) & 3];
            out++;
        } else if (type == 1) { /* insertion before p */
            uint32_t L = draw_run(sp, &r);
            for (uint32_t q = 0; q < L; q++) {
                uint8_t b = (uint8_t)BASES[rng_next(&r) >> 62];
                if (txt) txt[out] = b;
                out++;
            }
            if (txt) txt[out] = pat ? pat[p] : 0;
            out++;
        } else { /* deletion of p (and a run, stopped at the next event) */
            uint32_t L = draw_run(sp, &r);
            skip_until = p + L;
        }
    }
    *pn = n;
    *tm = out;
}

uint32_t synth_max_length(const synth_spec *sp) {
    return sp->len_dist == SYNTH_LEN_FIXED ? sp->n_lo : sp->n_hi;
}

int synth_lengths(const synth_spec *sp, uint64_t seed, uint64_t first, uint64_t count,
                  uint32_t *plen, uint32_t *tlen) {
    uint32_t nmax = synth_max_length(sp);
    uint64_t *mark = (uint64_t *)malloc((nmax / 64 + 1) * sizeof(uint64_t));
    if (!mark) return -1;
    for (uint64_t i = 0; i < count; i++)
        gen_pair(sp, seed, first + i, NULL, NULL, &plen[i], &tlen[i], mark);
    free(mark);
    return 0;
}

int synth_fill(const synth_spec *sp, uint64_t seed, uint64_t first, uint64_t count,
               const uint64_t *poff, const uint64_t *toff, uint8_t *pbuf, uint8_t *tbuf) {
    uint32_t nmax = synth_max_length(sp);
    uint64_t *mark = (uint64_t *)malloc((nmax / 64 + 1) * sizeof(uint64_t));
    if (!mark) return -1;
    for (uint64_t i = 0; i < count; i++) {
        uint32_t n, m;
        gen_pair(sp, seed, first + i, pbuf + poff[i], tbuf + toff[i], &n, &m, mark);
    }
    free(mark);
    return 0;
}
