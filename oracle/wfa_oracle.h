/* CPU oracle for gap-affine WFA alignment.  TEST INFRASTRUCTURE ONLY. */
#ifndef WFA_ORACLE_H
#define WFA_ORACLE_H
#include <stdint.h>

enum { ORACLE_OK = 0, ORACLE_E_INVAL = -1, ORACLE_E_NOMEM = -3, ORACLE_E_CAPACITY = -4 };

typedef struct {
    int64_t cells;       /* sum over score steps of wavefront widths          */
    int64_t steps;       /* score steps that hold a wavefront                 */
    int64_t ext_calls;   /* extend calls (non-NULL M cells)                   */
    int64_t ext_windows; /* 32-base windows an extend by word compare needs   */
    int64_t ext_matches; /* matching characters walked by extend              */
} oracle_stats;

int oracle_align(const uint8_t *P, int n, const uint8_t *T, int m,
                 int x, int o, int e, int want_cigar,
                 int32_t *score_out, uint32_t *runs, int64_t runs_cap, int64_t *nruns_out,
                 oracle_stats *st);

/* Ends-free alignment: at most pb / tb leading and pe / te trailing pattern /
 * text bases may stay unaligned at no cost (all zero: global alignment). */
int oracle_align_ends(const uint8_t *P, int n, const uint8_t *T, int m,
                      int x, int o, int e, int pb, int pe, int tb, int te, int want_cigar,
                      int32_t *score_out, uint32_t *runs, int64_t runs_cap, int64_t *nruns_out,
                      oracle_stats *st);

/* WF-adaptive heuristic (global alignment): once a wavefront holds at least
 * min_wavefront_length diagonals, diagonals at its ends farther from the end
 * cell than the closest one by more than max_distance_threshold are dropped
 * (min_wavefront_length 0: exact). */
int oracle_align_adaptive(const uint8_t *P, int n, const uint8_t *T, int m, int x, int o, int e,
                          int min_wavefront_length, int max_distance_threshold, int want_cigar,
                          int32_t *score_out, uint32_t *runs, int64_t runs_cap, int64_t *nruns_out,
                          oracle_stats *st);

int oracle_align_batch_adaptive(const uint8_t *pbuf, const uint64_t *poff, const uint32_t *plen,
                                const uint8_t *tbuf, const uint64_t *toff, const uint32_t *tlen,
                                int64_t count, int x, int o, int e, int min_wavefront_length,
                                int max_distance_threshold, int want_cigar, int32_t *scores,
                                uint32_t *runs, int64_t slot, int64_t *nruns, int32_t *status,
                                int threads, oracle_stats *st);

int oracle_align_batch_ends(const uint8_t *pbuf, const uint64_t *poff, const uint32_t *plen,
                            const uint8_t *tbuf, const uint64_t *toff, const uint32_t *tlen,
                            int64_t count, int x, int o, int e, int pb, int pe, int tb, int te,
                            int want_cigar, int32_t *scores, uint32_t *runs, int64_t slot,
                            int64_t *nruns, int32_t *status, int threads, oracle_stats *st);

int oracle_align_batch(const uint8_t *pbuf, const uint64_t *poff, const uint32_t *plen,
                       const uint8_t *tbuf, const uint64_t *toff, const uint32_t *tlen,
                       int64_t count, int x, int o, int e, int want_cigar,
                       int32_t *scores, uint32_t *runs, int64_t slot, int64_t *nruns,
                       int32_t *status, int threads, oracle_stats *st);

int64_t oracle_pack2bit(const uint8_t *seq, int64_t len, uint64_t *words, int64_t nwords);
#endif
