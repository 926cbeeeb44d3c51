/*
 * wfa.h - batched gap-affine global pair alignment with the wavefront
 * algorithm on AMD Instinct MI355X (gfx950).
 *
 * What is computed.  The paper aligns many independent read pairs with the
 * wavefront algorithm (Introduction and Methods: each pair is aligned
 * independently and one result per pair is written back).  The algorithm
 * is WFA (Marco-Sola, Moure, Moreto, Espinosa, Bioinformatics 37(4), 2021):
 * for a pattern P of n bases and a text T of m bases it returns the optimal
 * gap-affine score
 *
 *     score = min over global alignments of
 *             x * #mismatches + sum over maximal gap runs (o + e * length)
 *
 * (matches cost 0) and, in CIGAR mode, one optimal alignment.  Where
 * several alignments are optimal a fixed tie-break picks one: in a match
 * state, a mismatch on the same diagonal is preferred to the end of an
 * insertion, which is preferred to the end of a deletion; inside a gap,
 * opening from a match state is preferred to extending the gap.  Scores
 * and CIGARs are bit-identical across every schedule and launch shape the
 * library offers.
 *
 * Conventions.
 *   - Diagonal k = h - v, offset = h, where (v, h) aligns P[0..v) with
 *     T[0..h).
 *   - CIGAR runs are 32-bit words  len << 4 | op  with op
 *       WFA_OP_MATCH    (0, 'M'): P[v] == T[h], consumes one base of each;
 *       WFA_OP_MISMATCH (1, 'X'): P[v] != T[h], consumes one base of each;
 *       WFA_OP_INS      (2, 'I'): consumes one base of the TEXT only;
 *       WFA_OP_DEL      (3, 'D'): consumes one base of the PATTERN only.
 *     Neighbouring runs always have different ops.
 *   - Penalties: x = mismatch > 0, o = gap_open >= 0, e = gap_extend > 0.
 *
 * Sequence encodings.
 *   - WFA_ASCII:   bytes A, C, G, T (either case).  p_start / t_start are
 *                  byte offsets into `patterns` / `texts`.  Any other byte
 *                  makes the call fail with WFA_E_ALPHABET.
 *   - WFA_PACKED2: 2 bits per base in little-endian 64-bit words, A=0, C=1,
 *                  G=2, T=3; base i of a sequence sits in bits 2*(i%32) and
 *                  2*(i%32)+1 of word start + i/32.  p_start / t_start are
 *                  64-bit word indices.  Only the ceil(len/32) words of a
 *                  sequence are read; bits past its end are ignored.
 *
 * Memory spaces.  All buffer arguments of one call live in the space named
 * by `mem`: host memory (WFA_HOST) or device memory of the context's GPU
 * (WFA_DEVICE, e.g. torch tensors' data pointers).  Scalar out-parameters
 * (cigar_needed, bad_pair, stats, tickets) are always host pointers.
 * A host-memory batch runs as a pipeline over chunks of consecutive pairs:
 * while chunk i aligns, one library thread copies chunk i+1's descriptors
 * and sequence bytes to the device and another copies chunk i-1's scores,
 * offsets and runs back, each on a stream of its own.  Host buffers from
 * wfa_host_alloc (page-locked) move by DMA at the full link rate; ordinary
 * pageable buffers go through page-locked staging slots that library
 * threads fill and empty while the DMA engine moves the previous slot.
 *
 * Ownership.  The caller owns every input and output buffer; the library
 * keeps no caller pointer after a call returns.  The library owns its
 * device workspace, which grows on demand within the context's HBM budget.
 *
 * Synchronisation.  wfa_align_batch enqueues its work on `stream` (a
 * hipStream_t; NULL selects the context's own stream) and returns after that
 * work has completed.
 *
 * Threading.  A wfa_ctx is used by one host thread at a time.  The server
 * functions are thread-safe.
 *
 * Errors.  Every int-returning function returns WFA_OK (0) or a negative
 * WFA_E_* code; wfa_strerror gives its text.  On a validation error found on
 * the host (WFA_E_INVAL, WFA_E_CAPACITY's size check aside) nothing is
 * written except *bad_pair.  WFA_E_ALPHABET and WFA_E_TOO_LONG are found by
 * kernels, which may already have written scores, offsets and runs; their
 * contents are then unspecified.
 *
 * Plan reuse.  A call whose buffers (pointers), pair count, run capacity,
 * 2-bit packed input and settings equal the previous call's on the context
 * starts that call's launch before its batch facts are read back, and keeps
 * the results if the facts lead to the same plan; otherwise it runs again as
 * planned.  Results never depend on it.
 */
#ifndef WFA_H
#define WFA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wfa_ctx wfa_ctx;

typedef struct {
    int32_t mismatch;   /* x > 0  */
    int32_t gap_open;   /* o >= 0 */
    int32_t gap_extend; /* e > 0  */
} wfa_penalties;

/* One pair: start offsets (bytes for ASCII, 64-bit words for PACKED2) and
 * lengths.  24 bytes, naturally aligned. */
typedef struct {
    uint64_t p_start;
    uint64_t t_start;
    uint32_t p_len;
    uint32_t t_len;
} wfa_pair;

typedef enum { WFA_SCORE = 0, WFA_CIGAR = 1 } wfa_mode;
typedef enum { WFA_ASCII = 0, WFA_PACKED2 = 1 } wfa_encoding;
typedef enum { WFA_HOST = 0, WFA_DEVICE = 1 } wfa_memspace;

/* Schedules (all give identical results):
 *   AUTO:       persistent, bucketed, graph-replayed short-pair kernel, with
 *               the general kernel for pairs it cannot hold;
 *   PLAIN:      one launch, pair i on lane group i, no bucketing;
 *   PERSISTENT: grid sized to the GPU, lane groups pull pairs from a device
 *               queue in bucketed order;
 *   GENERAL:    every pair on the workgroup-per-pair kernel whose
 *               wavefronts live in the HBM arena (any length, any score). */
typedef enum {
    WFA_SCHED_AUTO = 0,
    WFA_SCHED_PLAIN = 1,
    WFA_SCHED_PERSISTENT = 2,
    WFA_SCHED_GENERAL = 3
} wfa_schedule;

/* Tuning knobs.  Zero means "choose automatically".  None of them changes
 * any result. */
typedef struct {
    int32_t schedule;       /* wfa_schedule                                      */
    int32_t window;         /* diagonals held per pair by the short kernel:
                               16, 24, 32, 48, 64, 128, 256 */
    int32_t step_cap;       /* score steps (in units of gcd(x,o,e)) held in LDS  */
    int32_t use_graph;      /* 1: the whole first pass (counters, packing,
                               bucketing, the short kernel, CIGAR offsets and
                               compaction) is captured once as a hipGraph and
                               replayed, one hipGraphLaunch per call;
                               2: the work before and after the short kernel
                               as two graphs, the kernel launched between them
                               (wfa_stats.ms_align then times the kernel alone);
                               -1: never; 0: form 1 for the persistent and
                               automatic schedules */
    int32_t bucket;         /* 1: sort pairs by (length, length difference); -1: off */
    int32_t general_pairs;  /* concurrent pairs of the general kernel; 0: by budget */
    int32_t block_threads;  /* threads per workgroup of the short kernel: 64..256 */
    int32_t lanes_per_pair; /* lanes of a wavefront per pair in the short kernel
                               (8, 16, 32 or 64, at most the window): 64 / lanes
                               pairs share a wavefront */
    int32_t host_chunk_pairs; /* pairs per chunk of the host-memory pipeline
                                 (at least 1/1024 of the batch); 0: a quarter
                                 of the batch, within [262144, 2097152] */
    int32_t cascade_window;   /* largest window of the cascade: further
                                 short-kernel passes, each over the pairs the
                                 previous pass handed over, with windows 64,
                                 128, 256 above the first; only what the last
                                 pass hands over goes to the general kernel.
                                 0: up to 256; -1: no cascade */
    int32_t general_slice_kib; /* CIGAR mode: first guess of the history bytes
                                 (KiB) per pair of the general kernel; a pair
                                 whose history outgrows its slice is re-run
                                 with a 4x slice.  0: estimated from the
                                 lengths and the history seen so far */
    int32_t lane_kernel;      /* 0 or 1: the first pass runs on the
                                 one-pair-per-lane kernel, whose wavefront rows
                                 live in registers, whenever it is built for the
                                 penalties (x, o, e = 4, 6, 2 and multiples),
                                 every sequence has at most 127 bases, the
                                 alignment is global, no window or lanes per
                                 pair are asked for and step_cap is at most 16
                                 (it holds 8 steps if step_cap <= 8, else 16);
                                 -1: never */
    int32_t general_step_limit; /* diagnostic: score steps (in units of
                                 gcd(x,o,e)) after which the general kernel
                                 gives up on a pair, which makes the call
                                 return WFA_E_LIMIT.  0: no limit below the
                                 bound that deleting all of P and inserting
                                 all of T implies, so only an internal error
                                 can give up */
    int32_t general_checkpoint; /* CIGAR mode of the general kernel: C in
                                 [1, 256] (raised to pre + 1, pre = max(x,
                                 o + e) in units of gcd(x, o, e)) keeps the
                                 wavefront rows of pre + 1 consecutive steps
                                 every C steps and
                                 recomputes the steps in between during the
                                 backtrace (far less memory per pair, the same
                                 CIGAR); -1 keeps a history row of every step;
                                 0: full history when the device memory holds
                                 it for every pair of the launch, checkpoints
                                 every 128 steps beyond */
} wfa_options;

/* Ends-free alignment.  Up to pattern_begin_free leading pattern bases OR
 * up to text_begin_free leading text bases, and up to pattern_end_free
 * trailing pattern bases OR up to text_end_free trailing text bases, may
 * stay unaligned at no cost (each bound is clipped to its sequence's length
 * per pair).  The score is the least gap-affine score over the allowed
 * starts and ends; the CIGAR still spells both sequences whole, the free
 * prefix and suffix as I (text) or D (pattern) runs (a free run and a paid
 * gap of the same op next to it share one run).  Of several optimal end
 * cells the one on the lowest diagonal (h - v) is taken.  All four zero:
 * global alignment.  Semi-global alignment of a read inside a reference is
 * text_begin_free = text_end_free = the text length. */
typedef struct {
    uint32_t pattern_begin_free;
    uint32_t pattern_end_free;
    uint32_t text_begin_free;
    uint32_t text_end_free;
} wfa_ends_free;

/* WF-adaptive heuristic: the wavefront reduction of the WFA paper that the
 * method builds on (Marco-Sola et al. 2021).  After each score step's
 * extension, a wavefront that spans at least min_wavefront_length diagonals
 * (those without an offset included) drops the diagonals at either end
 * whose furthest point (v, h) lies farther from the end cell than the
 * closest one by more than max_distance_threshold, the distance being
 * max(n - v, m - h), the bases still to cover (diagonals without an offset
 * count as farthest).  The step that reaches the end cell is never reduced.
 * The score is that of the path the search took, at least the optimum; the
 * CIGAR spells that path and may cost less than the score where the path
 * closes a gap and at once opens another of the same kind (one run in the
 * CIGAR, one opening cheaper).  min_wavefront_length 0 selects exact
 * alignment (the default). */
typedef struct {
    int32_t min_wavefront_length;
    int32_t max_distance_threshold;
} wfa_heuristic;

/* Counters of the last wfa_align_batch call on a context. */
typedef struct {
    uint64_t pairs;              /* pairs aligned                                    */
    uint64_t short_pairs;        /* pairs finished by the short-pair kernel          */
    uint64_t general_pairs;      /* pairs finished by the general kernel             */
    uint64_t requeued;           /* pairs re-run after exceeding a window, step or
                                    memory limit (results are unaffected)            */
    uint64_t cigar_runs;         /* total runs written                               */
    int32_t window;              /* short-kernel window used                         */
    int32_t lanes_per_pair;      /* short-kernel lanes per pair used                 */
    int32_t host_chunks;         /* chunks of the host-memory pipeline (0: device call) */
    int32_t step_cap;            /* short-kernel step cap used                       */
    int32_t schedule;            /* schedule used                                    */
    int32_t graph_replayed;      /* graph form used (wfa_options.use_graph): 0 none,
                                    1 one graph of the whole first pass, whose
                                    duration ms_align then holds, 2 graphs
                                    around a directly launched kernel        */
    double ms_pack;              /* device time of each phase, milliseconds          */
    double ms_align;
    double ms_general;
    double ms_compact;
    double ms_total;             /* host wall time of the call                       */
    int32_t cascade_window;      /* window of the cascade's last pass, 0: none       */
    int32_t lane_kernel;         /* 1 if the first pass ran one pair per lane
                                    (window 0, lanes_per_pair 1)               */
} wfa_stats;

enum {
    WFA_OK = 0,
    WFA_E_INVAL = -1,    /* bad argument: penalties, NULL pointer, enum value */
    WFA_E_ALPHABET = -2, /* a byte outside ACGTacgt (ASCII input)             */
    WFA_E_NOMEM = -3,    /* the HBM budget cannot hold the work; the context's
                            device workspace is then released, so that a later
                            batch that fits starts from nothing             */
    WFA_E_CAPACITY = -4, /* cigar_capacity is smaller than *cigar_needed      */
    WFA_E_DEVICE = -5,   /* a HIP call failed                                 */
    WFA_E_TOO_LONG = -6, /* a sequence longer than WFA_MAX_LENGTH             */
    WFA_E_BUSY = -7,     /* server queue full / ticket not finished          */
    WFA_E_NOTFOUND = -8, /* unknown server ticket                             */
    WFA_E_LIMIT = -9     /* the general kernel gave up on *bad_pair: more score
                            steps than wfa_options.general_step_limit, or a
                            history walk that did not lead back to the start
                            (an internal error); that pair's score is -1 and
                            the CIGAR outputs are not written               */
};

enum { WFA_OP_MATCH = 0, WFA_OP_MISMATCH = 1, WFA_OP_INS = 2, WFA_OP_DEL = 3 };

#define WFA_MAX_LENGTH ((uint32_t)1 << 26) /* bases per sequence */

/* Source: the host side of the paper's system (Introduction and Methods:
 * the host sets up the processing units that align the pairs); here one
 * context per GPU.
 * Create a context on HIP device `device` whose device workspace may grow to
 * `hbm_budget_bytes` (0: three quarters of the device's memory; the
 * workspace only grows as far as the batches need).  *out receives the
 * context. */
int wfa_ctx_create(int device, size_t hbm_budget_bytes, wfa_ctx **out);

/* Source: as wfa_ctx_create.
 * Free the context and all device memory it owns, including the engines
 * that closed servers left with it.  Every server opened on it must be
 * closed first.  NULL is ignored. */
void wfa_ctx_destroy(wfa_ctx *ctx);

/* Source: none in the paper (launch shape only; no result depends on it).
 * Set tuning knobs for later calls (NULL restores the defaults); a value
 * outside the documented ranges is WFA_E_INVAL and changes nothing. */
int wfa_set_options(wfa_ctx *ctx, const wfa_options *opt);

/* Source: a mode variant beyond the paper's global alignment (its Results
 * close with other alignment algorithms as future work); the score is the least
 * global score over the allowed clipped sub-pairs.
 * Select ends-free alignment (wfa_ends_free) for later wfa_align_batch and
 * wfa_autotune calls on the context, and for servers opened on it later
 * (a server keeps the setting it opened with); NULL or all zero selects
 * global alignment (the default).  Bounds above WFA_MAX_LENGTH are
 * WFA_E_INVAL. */
int wfa_set_ends_free(wfa_ctx *ctx, const wfa_ends_free *ends);

/* Source: the WF-adaptive heuristic of the WFA paper (Marco-Sola et al.
 * 2021) that Introduction and Methods builds on; a faster, inexact mode.
 * Select the heuristic (wfa_heuristic) for later wfa_align_batch,
 * wfa_align_batch_noalloc and wfa_autotune calls on the context, and for
 * servers opened on it later; NULL or min_wavefront_length 0 selects exact
 * alignment.  Every pair then runs on the general kernel.  The heuristic
 * applies to global alignment only: selecting it while free ends are set
 * (or free ends while it is selected), or a negative field, is
 * WFA_E_INVAL and changes nothing. */
int wfa_set_heuristic(wfa_ctx *ctx, const wfa_heuristic *h);

/* Source: Introduction and Methods -- every read pair is aligned on its own
 * with the wavefront algorithm (gap-affine WFA, Marco-Sola et al. 2021:
 * the I/D/M recurrences over diagonals, extension along matches, the end
 * at M_s[m - n] = m, and the backtrace) and one result per pair is written
 * back; Results -- 5 M pairs of 100 bp per batch.
 * Align num_pairs pairs.
 *   patterns, texts   sequence buffers in `enc` and `mem`
 *   pairs             [num_pairs] descriptors, in `mem`
 *   pen, mode         penalties and result mode
 *   scores            [num_pairs] int32 out, in `mem`
 *   cigar_runs        runs out (CIGAR mode; NULL allowed with capacity 0)
 *   cigar_capacity    number of uint32 words cigar_runs can hold
 *   cigar_offsets     [num_pairs + 1] uint64 out (CIGAR mode): pair i's runs
 *                     are cigar_runs[cigar_offsets[i] .. cigar_offsets[i+1])
 *   cigar_needed      host out: total runs of all pairs (may be NULL)
 *   bad_pair          host out: first pair that failed validation, else -1
 *   stream            hipStream_t or NULL
 * In WFA_SCORE mode the CIGAR arguments are ignored.  If cigar_capacity is
 * too small the call returns WFA_E_CAPACITY after writing scores, offsets
 * and *cigar_needed; the runs can then be fetched with wfa_copy_last_cigars.
 */
int wfa_align_batch(wfa_ctx *ctx, const void *patterns, const void *texts,
                    const wfa_pair *pairs, size_t num_pairs, wfa_encoding enc,
                    wfa_memspace mem, wfa_penalties pen, wfa_mode mode, int32_t *scores,
                    uint32_t *cigar_runs, size_t cigar_capacity, uint64_t *cigar_offsets,
                    size_t *cigar_needed, int64_t *bad_pair, void *stream);

/* Source: as wfa_align_batch (the results written back).
 * After WFA_E_CAPACITY: copy the runs of the last call into `runs` (in the
 * last call's memory space) if `capacity` suffices; offsets are those the
 * last call wrote and may be passed again (NULL: not rewritten). */
int wfa_copy_last_cigars(wfa_ctx *ctx, uint32_t *runs, size_t capacity, uint64_t *offsets);

/* Source: Results -- the paper's `Total` time includes moving pairs and
 * results between the host and the processing units, which dominated it.
 * Page-locked host memory for WFA_HOST batches (inputs and outputs), so
 * that the host-memory pipeline's copies run at the full link rate.
 * hipHostMalloc underneath: *out receives `bytes` bytes (0 is allowed and
 * gives a valid pointer) or NULL with WFA_E_NOMEM.  The caller owns the
 * block until wfa_host_free; it is not tied to a context.  */
int wfa_host_alloc(size_t bytes, void **out);

/* Source: as wfa_host_alloc.  Free a block from wfa_host_alloc.  NULL is
 * ignored. */
void wfa_host_free(void *ptr);

/* Source: Introduction and Methods -- the sequences of a pair are fetched
 * into fast local memory before alignment; here they are read as 2-bit
 * packed words.
 * Encode ASCII sequences to the PACKED2 layout on the device.
 *   ascii        device bytes
 *   starts/lens  [count] device arrays: byte offset and length per sequence
 *   words        device output; sequence i starts at word word_starts[i]
 *   word_starts  [count + 1] device out: exclusive scan of ceil(len/32),
 *                the last entry being the total
 *   total_words  host out: words written
 *   bad_index    host out: sequence index of the first non-ACGT byte, or -1
 * Fails with WFA_E_ALPHABET if any byte is outside ACGTacgt; WFA_E_CAPACITY
 * if `words_capacity` is smaller than the words needed. */
int wfa_pack2bit(wfa_ctx *ctx, const uint8_t *ascii, const uint64_t *starts,
                 const uint32_t *lens, size_t count, uint64_t *words, size_t words_capacity,
                 uint64_t *word_starts, size_t *total_words, int64_t *bad_index, void *stream);

/* Source: none in the paper (the launch shape is picked by measurement; no
 * result depends on it).
 * Autotuner.  Times candidate options on the
 * first `sample_pairs` pairs (0: 262144) of the given batch, in two stages:
 * first every first-pass shape -- the one-pair-per-lane kernel where it is
 * built for the penalties and lengths (step cap 8 if the sample's largest
 * score step allows, else 16), and every short-kernel shape (window, lanes
 * per pair) whose window can hold the sample's length differences -- on the
 * plain schedule, plus the general kernel; then, for the two fastest shapes,
 * every workgroup size (64, 128, 256), schedule form (plain; persistent with
 * and without bucketing) and step cap (the default, and the largest score
 * step of the sample, found by a score-only pass); the library's own default
 * choice is always a candidate.  A candidate's time is the fastest of several
 * calls.  Every candidate must return byte-identical results; the fastest is
 * applied to the context and cached in the JSON file `cache_path` (NULL: no
 * cache) under a key of device architecture, penalties, mode and the batch's
 * length / length-difference / size classes; a later call with the same key
 * reuses it unless `force` is set.  Arguments as wfa_align_batch; *chosen
 * receives the options.  WFA_E_DEVICE if two candidates disagree. */
int wfa_autotune(wfa_ctx *ctx, const void *patterns, const void *texts, const wfa_pair *pairs,
                 size_t num_pairs, wfa_encoding enc, wfa_memspace mem, wfa_penalties pen,
                 wfa_mode mode, size_t sample_pairs, const char *cache_path, int force,
                 wfa_options *chosen);

/* ---------------------------------------------------------------------------
 * Allocation-free alignment.
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments and results as wfa_align_batch with mem = WFA_DEVICE (every
 * buffer is device memory the caller owns), the context's options and free
 * ends, but graphs are never captured, and the call allocates no device
 * memory: its whole workspace (batch statistics, counters, packed sequences,
 * CIGAR slots, bucketing, the cascade and the general kernel's arena) is
 * carved from a static device array of WFA_NOALLOC_SCRATCH_BYTES that each
 * GPU the library runs on holds until the process ends.  Limits and errors:
 *   - num_pairs above WFA_NOALLOC_MAX_PAIRS: WFA_E_INVAL, nothing written;
 *   - a workspace larger than the array (long or very divergent pairs whose
 *     general-kernel slices do not fit): WFA_E_NOMEM;
 *   - WFA_E_CAPACITY: scores, offsets and *cigar_needed are written, but the
 *     runs are not kept for wfa_copy_last_cigars (call again with room).
 * Every call on a GPU, from any context, uses that GPU's one array: calls
 * that overlap in time on one GPU race and must be serialised by the caller.
 * Each call clears whatever it relies on; nothing carries over between calls.
 * ------------------------------------------------------------------------- */
#define WFA_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
#define WFA_NOALLOC_MAX_PAIRS ((uint32_t)1 << 18)

int wfa_align_batch_noalloc(wfa_ctx *ctx, const void *patterns, const void *texts,
                            const wfa_pair *pairs, size_t num_pairs, wfa_encoding enc,
                            wfa_penalties pen, wfa_mode mode, int32_t *scores,
                            uint32_t *cigar_runs, size_t cigar_capacity,
                            uint64_t *cigar_offsets, size_t *cigar_needed, int64_t *bad_pair,
                            void *stream);

/* Source: Results -- the paper reports `Kernel` and `Total` time apart;
 * these are the device time of each phase and the call's wall time.
 * Counters of the last wfa_align_batch call. */
int wfa_last_stats(const wfa_ctx *ctx, wfa_stats *out);

/* Source: none in the paper.  Text of a status code (static storage). */
const char *wfa_strerror(int status);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of alignment requests.
 *
 * Requests (each a set of pairs) are submitted from any thread and get a
 * ticket.  One worker per stream forms a batch whenever it is free: it takes
 * pending pairs in arrival order -- the rest of a request already running,
 * then whole or partial later requests -- while the batch stays under
 * max_chunk_pairs and the estimated device memory of everything admitted
 * stays under the budget.  Batches of different workers run concurrently on
 * their own streams, so requests that arrive while others are on the GPU
 * join as soon as a worker and memory free up.  A request completes when its
 * last pair does.  Results equal those of wfa_align_batch on the same pairs
 * alone: every pair is aligned independently and deterministically.
 * Source: the paper aligns one offline batch; serving many requests with
 * continuous batching rests on the same per-pair independence (Introduction
 * and Methods).
 * ------------------------------------------------------------------------- */
typedef struct wfa_server wfa_server;

/* A request: host ASCII sequences (p_start / t_start are byte offsets into
 * `patterns` / `texts`).  wfa_server_submit copies everything it needs. */
typedef struct {
    const uint8_t *patterns;
    const uint8_t *texts;
    const wfa_pair *pairs;
    size_t num_pairs;
} wfa_request;

/* Optional replacement for the GPU engine (used to test the scheduler on a
 * CPU, or to plug in another executor).  It aligns one merged batch in host
 * memory with the server's penalties and mode and returns a WFA_* status;
 * `runs` holds `capacity` words, *needed receives the runs required. */
typedef int (*wfa_executor_fn)(void *user, const wfa_request *batch, int32_t *scores,
                               uint32_t *runs, size_t capacity, uint64_t *offsets,
                               size_t *needed);

typedef struct {
    size_t hbm_budget_bytes;   /* admission budget (0: 64 GiB)                   */
    int32_t streams;           /* concurrent device streams, one worker each (0: 4) */
    int32_t max_chunk_pairs;   /* pairs per launched batch (0: 65536)            */
    int32_t queue_limit;       /* requests waiting for admission (0: 1 << 20)     */
    int32_t mode;              /* wfa_mode for every request                     */
    wfa_penalties pen;
    wfa_executor_fn executor;  /* NULL: the GPU engine of `ctx`                  */
    void *executor_user;
} wfa_server_cfg;

/* A finished request: host arrays owned by the server until the ticket is
 * released (wfa_server_release) or the server closes. */
typedef struct {
    size_t num_pairs;
    const int32_t *scores;
    const uint32_t *cigar_runs;
    const uint64_t *cigar_offsets; /* [num_pairs + 1] (CIGAR mode)               */
    double submit_time_s;          /* seconds since the server opened            */
    double admit_time_s;           /* first pair admitted to the device          */
    double done_time_s;            /* last pair finished                         */
    int32_t status;                /* WFA_OK or the error of a batch it was in   */
} wfa_result;

typedef struct {
    uint64_t submitted, completed, batches, pairs;
    size_t budget_bytes;
    size_t reserved_bytes;       /* reserved now                                  */
    size_t max_reserved_bytes;   /* high-water mark (never above budget_bytes,
                                    except a lone request larger than the budget) */
    double busy_s;               /* summed engine time                            */
} wfa_server_stats;

/* Open a server on `ctx` (which must outlive it; NULL only with an executor).
 * Each stream gets its own device workspace of budget/streams bytes. */
int wfa_server_open(wfa_ctx *ctx, const wfa_server_cfg *cfg, wfa_server **out);
/* Queue a request; *ticket identifies it.  WFA_E_BUSY if the queue is full. */
int wfa_server_submit(wfa_server *srv, const wfa_request *req, uint64_t *ticket);
/* Wait up to timeout_us (negative: forever) for a ticket.  Returns WFA_OK and
 * fills *out, WFA_E_BUSY on time-out, WFA_E_NOTFOUND for an unknown ticket. */
int wfa_server_poll(wfa_server *srv, uint64_t ticket, int64_t timeout_us, wfa_result *out);
/* Free a finished request's results. */
int wfa_server_release(wfa_server *srv, uint64_t ticket);
/* Device bytes the admission controller reserves for a request: staged
 * sequences and results plus the wavefront memory of each pair (a ring of
 * full-width rows, and in CIGAR mode an O(s^2) history) with s the score
 * its length would have at 6 % divergence. */
size_t wfa_server_estimate_bytes(const wfa_server *srv, const wfa_request *req);
int wfa_server_get_stats(const wfa_server *srv, wfa_server_stats *out);
/* Finish all submitted work, stop the workers and free the server.  Its
 * per-stream engines (streams and device workspaces, up to 16 of them) stay
 * with the context and are taken over by the next server opened on it;
 * wfa_ctx_destroy frees them. */
int wfa_server_close(wfa_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* WFA_H */
