// Internal launch interface between the C-ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wfa {

// Same layout as the public wfa_pair.
struct PairDesc {
    uint64_t p_start;
    uint64_t t_start;
    uint32_t p_len;
    uint32_t t_len;
};

// Batch-wide facts gathered on the device before planning.
struct BatchStats {
    uint32_t max_p;
    uint32_t max_t;
    uint32_t max_absdiff;
    uint32_t too_long;
    uint64_t words_p;  // sum of ceil(p_len / 32)
    uint64_t words_t;
    uint64_t first_too_long;  // lowest pair index over the length limit, or ~0
};

// Blocks of the first batch-statistics pass; the statistics buffer holds
// 1 + STATS_BLOCKS records (result, then the partials).
constexpr int STATS_BLOCKS = 1024;

// Largest pre + 1 (rows a step reads back, plus the current one) the kernels hold.
constexpr int GENERAL_MAX_RING = 512;
// Checkpoint CIGAR mode of the general kernel: at most this many steps
// between checkpoints, and rows per recomputed segment (steps between two
// checkpoints plus the pre + 1 rows of a checkpoint)
constexpr int GENERAL_CKPT_MAX = 256;
constexpr int GENERAL_SEG_ROWS = 768;

// Penalties divided by their gcd g: every reachable score is a multiple of g,
// so the kernels step s' = s / g and report g * s'.
struct Pen {
    int x, oe, e;  // x/g, (o+e)/g, e/g
    int g;
    int pre;       // max(x, oe, e): rows a step reads back
};

// Ends-free alignment: at most pb / tb leading and pe / te trailing pattern /
// text bases stay unaligned at no cost (each clipped to its sequence's
// length per pair); all zero is global alignment.
struct Ends {
    int pb, pe, tb, te;
};

// WF-adaptive heuristic (the WFA paper's wavefront reduction; global
// alignment only): after a step's extension, a wavefront spanning at least
// mwl diagonals drops the diagonals at either end whose distance to the end
// cell, max(n - v, m - h), exceeds the least such distance by more than mdt.
// mwl = 0: exact alignment.
struct Heuristic {
    int mwl, mdt;
};

// Arguments of the short-pair kernel (all device pointers).
struct ShortArgs {
    const PairDesc* pairs;
    const uint64_t* pw;         // packed pattern words
    const uint64_t* tw;         // packed text words
    const uint32_t* order;      // queue position -> pair index (NULL: identity)
    uint32_t num;               // pairs in the queue
    uint32_t npairs;            // pairs of the batch (bound of the indices in `order`)
    Ends ends;                  // free ends (all zero: global alignment)
    uint32_t* queue;            // persistent: next queue position (device counter)
    int queue_chunk;            // rounds of 64/G pairs a wave claims per atomic
    Pen pen;
    int cap;                    // last step s' held
    int ring;                   // M rows: a ring of pre + 1 (score), or cap + 2 (CIGAR)
    int ring2;                  // I and D rows: rings of e + 1
    int id_off;                 // LDS byte offset of the I rows (the D rows follow)
    int seq_words;              // 64-bit words of LDS per sequence
    int group_bytes;            // LDS bytes per lane group
    int rows_bytes;             // LDS bytes of all offset rows (the I/D rings also stage runs)
    int slot_cap;               // most runs a pair may have in the kernel
    int row_bytes;              // 1: int8 offsets (sequences < 128 bases), 2: int16
    int32_t* scores;            // [pairs]
    uint32_t* nruns;            // [pairs] runs written
    uint64_t* run_src;          // [pairs] where the reversed runs live
    uint64_t run_src_add;       // added to run_src (a cascade pass: SLOTS2_BIT + its offset in slots2)
    uint32_t* slots;            // [pairs * slot_cap] reversed runs, packed per wave
    uint32_t* ovf_list;         // pairs the kernel could not hold
    uint32_t* ovf_count;
};

// Arguments of the one-lane-per-pair kernel (all device pointers).
struct LaneArgs {
    const PairDesc* pairs;
    const uint64_t* pw;         // packed pattern words
    const uint64_t* tw;         // packed text words
    const uint32_t* order;      // queue position -> pair index (NULL: identity)
    uint32_t num;               // pairs in the queue
    uint32_t npairs;            // pairs of the batch (bound of the indices in `order`)
    uint32_t* queue;            // persistent: LANE_QUEUES claim counters, 32 words apart
    Pen pen;
    int slot_cap;               // most runs a pair may have (CIGAR)
    int32_t* scores;            // [pairs]
    uint32_t* nruns;            // [pairs] runs written
    uint64_t* run_src;          // [pairs] where the reversed runs live (packed per group of 64)
    uint32_t* slots;            // [pairs * slot_cap] reversed runs
    uint32_t* hist;             // CIGAR: one history and run-stage region per launched wavefront
    uint32_t* ovf_list;         // pairs the kernel could not hold
    uint32_t* ovf_count;
};

// What the general kernel's forward pass hands to its CIGAR walk, per job.
struct GenJobState {
    long long bump;     // end of the history rows (or checkpoints) in the slice
    long long end_off;  // ring offset of the last step's rows
    int S;              // score steps of the alignment (-1: no walk)
    int end_k;          // diagonal of the end cell
};

// Arguments of the general (workgroup-per-pair, HBM arena) kernel.
struct GeneralArgs {
    const PairDesc* pairs;
    const uint64_t* pw;
    const uint64_t* tw;
    const uint32_t* jobs;       // pair index per workgroup
    uint32_t num_jobs;
    Pen pen;
    Ends ends;
    int cigar;
    uint8_t* arena;             // num_jobs slices, job j's at [slice_off[j], slice_off[j + 1])
    const uint64_t* slice_off;  // [num_jobs + 1] byte offsets of the slices
    int32_t* scores;
    uint32_t* nruns;
    uint64_t* run_src;          // offset (in uint32 words) of the job's runs in the arena
    uint32_t* job_nruns;        // [num_jobs] runs of each finished job (0 if it failed)
    uint64_t* job_used;         // [num_jobs] CIGAR mode: slice bytes past the ring a
                                // finished job used (history, step table, runs)
    uint32_t* fail_list;        // jobs whose slice was too small
    uint32_t* fail_count;
    // A pair the kernel gives up on -- more score steps than `step_limit`
    // (0: the bound n + m gap bases imply), or a history walk that does not
    // lead back to the origin -- gets score -1 and no runs, and the lowest
    // such pair index is kept here (atomicMin; the host starts it at ~0).
    unsigned long long* gave_up;
    long long step_limit;
    Heuristic heur;             // mwl = 0: exact
    // CIGAR mode: 0 keeps a history row of every step; C > 0 keeps the rows
    // of pre + 1 consecutive steps every C steps and recomputes the rest
    // during the backtrace (C <= GENERAL_CKPT_MAX, C + pre + 1 <=
    // GENERAL_SEG_ROWS)
    int ckpt;
    GenJobState* jstate;        // CIGAR mode: [num_jobs] hand-over to the walk kernel
};

// Kernel entry points (host-side launchers; all asynchronous on `s`).
hipError_t launch_batch_stats(const PairDesc* pairs, size_t n, BatchStats* out, uint32_t max_len,
                              hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s);
// Several fills in one launch: p[0..n) = v for each of up to FILL_OPS ranges
// (the ranges must not overlap).
constexpr int FILL_OPS = 8;
struct FillOp {
    uint32_t* p;
    uint64_t n;
    uint32_t v;
};
struct FillOps {
    FillOp op[FILL_OPS];
    int count = 0;
    void add(uint32_t* p, uint64_t n, uint32_t v) {  // a count past FILL_OPS fails the launch
        if (!n) return;
        if (count < FILL_OPS) op[count] = FillOp{p, n, v};
        count++;
    }
};
hipError_t launch_fill_multi(const FillOps& ops, hipStream_t s);
// dst[i] = src[i] + add for i < n
hipError_t launch_add_u64(const uint64_t* src, uint64_t add, size_t n, uint64_t* dst,
                          hipStream_t s);

// Exclusive scan: out[i] = sum_{j<i} in(j), out[n] = total.  `in` selects a
// per-pair quantity through `kind`.
enum ScanKind { SCAN_WORDS_P = 0, SCAN_WORDS_T = 1, SCAN_U32 = 2, SCAN_WORDS_LEN = 3 };
size_t scan_temp_bytes(size_t n);
hipError_t launch_scan(ScanKind kind, const void* in, size_t n, uint64_t* out, void* temp,
                       hipStream_t s);

// ASCII -> PACKED2 for both sides of `pairs` (word starts from the scans of
// ceil(len/32)), writing descriptors with word starts into packed_pairs.
// Sets *err_pair to the lowest pair index holding a non-ACGT byte
// (initialise to UINT64_MAX).
// ASCII pairs -> 2-bit words and word-start descriptors.  A side whose
// word-start array is NULL is laid out at a fixed stride of its max words.
hipError_t launch_pack_pairs(const PairDesc* pairs, size_t n, const uint8_t* pascii,
                             const uint8_t* tascii, const uint64_t* ws_p, const uint64_t* ws_t,
                             uint32_t max_words_p, uint32_t max_words_t, uint64_t* words_p,
                             uint64_t* words_t, PairDesc* packed_pairs, unsigned long long* err_pair,
                             hipStream_t s);
// ASCII -> PACKED2 for independent sequences (public wfa_pack2bit);
// word_starts[0..n] is the exclusive scan of ceil(len/32), total_words its end.
hipError_t launch_pack_seqs(const uint8_t* ascii, const uint64_t* starts, const uint32_t* lens,
                            size_t n, const uint64_t* word_starts, uint64_t total_words,
                            uint64_t* words, unsigned long long* err_index, hipStream_t s);

// Short-pair kernel: a window of `window` diagonals held by `lanes` lanes per
// pair (window / lanes diagonals per lane); see short_shape_supported.
bool short_shape_supported(int window, int lanes);
hipError_t launch_short(const ShortArgs& a, int window, int lanes, bool cigar, bool persistent,
                        int block_threads, int grid, hipStream_t s);
int short_groups_per_block(int lanes, int block_threads);
int short_max_blocks_per_cu(int window, int lanes, bool cigar, int block_threads,
                            int lds_per_block, int row_bytes);

// Claim counters of the persistent one-lane-per-pair kernel (each on its own
// 128-byte line: LANE_QUEUES * 32 words, zeroed before a launch).
constexpr int LANE_QUEUES = 64;

// One-lane-per-pair kernel: built for some scaled penalty sets and step caps
// (lane_supported); kmax is the largest |target diagonal| it can end on.
bool lane_supported(const Pen& pen, int cap, uint32_t max_len);
int lane_kmax(const Pen& pen, int cap);
int lane_lds_bytes(const Pen& pen, int cap, bool cigar, int block_threads);
int lane_max_blocks_per_cu(const Pen& pen, int cap, bool cigar, int block_threads);
// CIGAR history and run stage bytes of one wavefront (global memory, one
// region per wavefront of the launch)
size_t lane_hist_bytes_per_wave(const Pen& pen, int cap, bool cigar, int slot_cap);
hipError_t launch_lane(const LaneArgs& a, int cap, bool cigar, bool persistent, int block_threads,
                       int grid, hipStream_t s);

// rows16: 16-bit ring rows (every text of the launch shorter than 32767 bases)
hipError_t launch_general(const GeneralArgs& a, int block_threads, bool seq_in_lds,
                          int lds_bytes, bool rows16, hipStream_t s);

// Copy reversed runs from their staging places into the caller's buffer.
// Nothing is written if offsets[n] exceeds `capacity`.
// run_src of a pair: a word offset into `slots`, into `slots2` with
// SLOTS2_BIT set, or into `gen_runs` with GEN_BIT set
constexpr uint64_t GEN_BIT = 1ULL << 63;
constexpr uint64_t SLOTS2_BIT = 1ULL << 62;
// total_out (may be null) receives offsets[n], the run total, whether or not
// it fits the capacity.
hipError_t launch_compact(const uint64_t* run_src, const uint32_t* slots, const uint32_t* slots2,
                          const uint32_t* gen_runs, const uint64_t* offsets, size_t n,
                          uint32_t* out, uint64_t capacity, uint64_t* total_out, hipStream_t s);

// Counting sort of pairs by expected work: keys + histogram, then the
// scatter into `order` (each block takes the exclusive scan of the histogram
// itself and reserves its ranges through `taken`).  `hist` and `taken`
// (BUCKET_KEYS words each) must be zero before the keys kernel.
constexpr int BUCKET_KEYS = 4096;
hipError_t launch_bucket_keys(const PairDesc* pairs, size_t n, uint32_t* keys, uint32_t* hist,
                              hipStream_t s);
hipError_t launch_bucket_scatter(const uint32_t* keys, size_t n, const uint32_t* hist,
                                 uint32_t* taken, uint32_t* order, hipStream_t s);
// Gather runs of finished general jobs from the arena into gen_runs.
// out[2i], out[2i+1] = lengths of pair idx[i] (pattern, text)
hipError_t launch_pair_lengths(const PairDesc* pairs, const uint32_t* idx, size_t n, uint32_t* out,
                               hipStream_t s);
hipError_t launch_gather_general(const uint32_t* jobs, size_t njobs, const uint32_t* nruns,
                                 uint64_t* run_src, const uint8_t* arena, uint64_t slice_bytes,
                                 const uint64_t* job_offsets, uint64_t gen_base,
                                 uint32_t* gen_runs, hipStream_t s);
hipError_t launch_scatter_scores_fail(const uint32_t* list, size_t n, int32_t* scores,
                                      hipStream_t s);

}  // namespace wfa
