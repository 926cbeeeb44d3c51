/* Seeded synthetic read-pair generator (input bytes only; no alignment logic). */
#ifndef SYNTH_H
#define SYNTH_H
#include <stdint.h>

enum { SYNTH_LEN_FIXED = 0, SYNTH_LEN_UNIFORM = 1, SYNTH_LEN_LOGUNIFORM = 2 };
enum { SYNTH_EDITS_FIXED = 0, SYNTH_EDITS_RATE = 1 };

typedef struct {
    int32_t len_dist;   /* SYNTH_LEN_*                                   */
    uint32_t n_lo;      /* fixed length, or lower bound                  */
    uint32_t n_hi;      /* upper bound (uniform / log-uniform)           */
    int32_t edit_mode;  /* SYNTH_EDITS_*                                 */
    uint32_t edits;     /* event count when edit_mode == FIXED           */
    double r_lo, r_hi;  /* event rate range when edit_mode == RATE       */
    int32_t runs;       /* 0: single-base indels; 1: geometric(1/2) runs */
} synth_spec;

uint32_t synth_max_length(const synth_spec *sp);
/* Lengths of pairs [first, first+count). Returns 0, or -1 on allocation failure. */
int synth_lengths(const synth_spec *sp, uint64_t seed, uint64_t first, uint64_t count,
                  uint32_t *plen, uint32_t *tlen);
/* Bytes of the same pairs, written at pbuf+poff[i] and tbuf+toff[i]. */
int synth_fill(const synth_spec *sp, uint64_t seed, uint64_t first, uint64_t count,
               const uint64_t *poff, const uint64_t *toff, uint8_t *pbuf, uint8_t *tbuf);
#endif
