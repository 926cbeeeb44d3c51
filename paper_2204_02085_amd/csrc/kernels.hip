// HIP kernels for batched gap-affine WFA on gfx950 (CDNA4, wave64).
//
// Method: the wavefront algorithm (Marco-Sola et al., Bioinformatics 2021),
// which the paper runs per read pair (Introduction and Methods).  For a
// pattern P (n bases) and a text T (m bases), diagonal k = h - v and offset h:
//   I_s[k] = max{M_{s-o-e}[k-1] + 1, I_{s-e}[k-1] + 1}
//   D_s[k] = max{M_{s-o-e}[k+1],     D_{s-e}[k+1]}
//   M_s[k] = max{M_{s-x}[k] + 1, I_s[k], D_s[k]},  then extend M_s[k]
// A candidate offset c on diagonal k counts only if it is a real cell,
// c <= m and c - k <= n; the alignment ends at the first s with
// M_s[m-n] == m.  Scores step in units of g = gcd(x, o, e).
//
// Kernels:
//   k_batch_stats   lengths and word counts of a batch (planning)
//   k_fill_*        fills (one launch for several ranges: k_fill_multi)
//   k_scan_*        exclusive scan (word starts, CIGAR offsets, job offsets)
//   k_bucket_*      counting sort of pairs by expected work
//   k_pack_*        ASCII -> 2-bit little-endian words, alphabet check
//   k_short         short pairs: a lane group owns a fixed window of
//                   diagonals (one or more per lane); all wavefront rows of a
//                   pair live in LDS; one lane walks the backtrace
//   k_general       any pair: one workgroup per pair, wavefront rows in a
//                   per-pair slice of the HBM arena
//   k_compact       reversed per-pair runs -> caller's CIGAR buffer
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace wfa {

namespace {

constexpr int NUL16 = -16384;          // NULL offset in int16 rows
constexpr int NUL32 = -(1 << 30);      // NULL offset in int32 rows
enum { OP_M = 0, OP_X = 1, OP_I = 2, OP_D = 3 };

__device__ __forceinline__ void wave_sync() {
    // LDS traffic of one wave executes in order; this only stops the compiler
    // from moving LDS accesses across a hand-off between lanes.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 32 bases starting at base `pos` of a 2-bit little-endian sequence held as
// 32-bit words S[] (16 bases each); dwords S[pos/16 .. pos/16 + 2] must exist.
// Pointers into LDS typed as such, so their arithmetic stays 32-bit.
template <class T>
using lds_ptr = __attribute__((address_space(3))) T*;

template <class P>
__device__ __forceinline__ uint64_t window32(P S, int pos) {
    const int q = pos >> 4;
    const uint32_t b = (uint32_t)(pos & 15) << 1;
    const uint32_t w0 = S[q], w1 = S[q + 1], w2 = S[q + 2];
    const uint32_t lo = __builtin_amdgcn_alignbit(w1, w0, b);
    const uint32_t hi = __builtin_amdgcn_alignbit(w2, w1, b);
    return ((uint64_t)hi << 32) | lo;
}

// Matching bases at the start of two windows (32 if all match).
__device__ __forceinline__ int common_prefix(uint64_t a, uint64_t b) {
    const uint64_t d = a ^ b;
    return d ? (__builtin_ctzll(d) >> 1) : 32;
}

__device__ __forceinline__ uint32_t cdiv32(uint32_t a) { return (a + 31u) >> 5; }

// ---------------------------------------------------------------------------
// planning
// ---------------------------------------------------------------------------
// Two passes without atomics: every block reduces a grid-strided share of the
// pairs into its own partial, then one block reduces the partials.
__device__ __forceinline__ void stats_reduce_block(BatchStats& v, BatchStats* out) {
    for (int off = 32; off > 0; off >>= 1) {
        v.max_p = max(v.max_p, (uint32_t)__shfl_xor((int)v.max_p, off));
        v.max_t = max(v.max_t, (uint32_t)__shfl_xor((int)v.max_t, off));
        v.max_absdiff = max(v.max_absdiff, (uint32_t)__shfl_xor((int)v.max_absdiff, off));
        v.too_long |= (uint32_t)__shfl_xor((int)v.too_long, off);
        v.words_p += __shfl_xor(v.words_p, off);
        v.words_t += __shfl_xor(v.words_t, off);
        v.first_too_long = min(v.first_too_long, (uint64_t)__shfl_xor(v.first_too_long, off));
    }
    __shared__ BatchStats sh[4];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); w++) {
            v.max_p = max(v.max_p, sh[w].max_p);
            v.max_t = max(v.max_t, sh[w].max_t);
            v.max_absdiff = max(v.max_absdiff, sh[w].max_absdiff);
            v.too_long |= sh[w].too_long;
            v.words_p += sh[w].words_p;
            v.words_t += sh[w].words_t;
            v.first_too_long = min(v.first_too_long, sh[w].first_too_long);
        }
        *out = v;
    }
}

__global__ __launch_bounds__(256) void k_batch_stats(const PairDesc* __restrict__ pairs, size_t n,
                                                     BatchStats* __restrict__ partial,
                                                     uint32_t max_len) {
    BatchStats v{0u, 0u, 0u, 0u, 0ull, 0ull, ~0ull};
    const size_t stride = (size_t)gridDim.x * blockDim.x;
#pragma unroll 4
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t p = pairs[i].p_len, t = pairs[i].t_len;
        v.max_p = max(v.max_p, p);
        v.max_t = max(v.max_t, t);
        v.max_absdiff = max(v.max_absdiff, p > t ? p - t : t - p);
        const bool tl = p > max_len || t > max_len;
        v.too_long |= tl ? 1u : 0u;
        v.first_too_long = tl ? min(v.first_too_long, (uint64_t)i) : v.first_too_long;
        v.words_p += cdiv32(p);
        v.words_t += cdiv32(t);
    }
    stats_reduce_block(v, partial + blockIdx.x);
}

__global__ __launch_bounds__(256) void k_batch_stats_final(const BatchStats* __restrict__ partial,
                                                           int nb, BatchStats* __restrict__ out) {
    BatchStats v{0u, 0u, 0u, 0u, 0ull, 0ull, ~0ull};
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const BatchStats q = partial[b];
        v.max_p = max(v.max_p, q.max_p);
        v.max_t = max(v.max_t, q.max_t);
        v.max_absdiff = max(v.max_absdiff, q.max_absdiff);
        v.too_long |= q.too_long;
        v.words_p += q.words_p;
        v.words_t += q.words_t;
        v.first_too_long = min(v.first_too_long, q.first_too_long);
    }
    stats_reduce_block(v, out);
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// dst[i] = src[i] + add: a chunk's offsets, counted from its first run, made
// relative to the first run of the whole batch
__global__ void k_add_u64(const uint64_t* __restrict__ src, uint64_t add, size_t n,
                          uint64_t* __restrict__ dst) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i] + add;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// One launch for several fills.  Every thread walks the ranges in turn (the
// loop over ranges is uniform), storing four words at a time where a range
// starts on a 16-byte boundary.
__global__ __launch_bounds__(256) void k_fill_multi(FillOps ops) {
    const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (int o = 0; o < ops.count; o++) {
        uint32_t* p = ops.op[o].p;
        const uint64_t n = ops.op[o].n;
        const uint32_t v = ops.op[o].v;
        uint64_t head = 0;
        if (((uintptr_t)p & 15) == 0) {
            const uint64_t n4 = n / 4;
            const uint4 w = make_uint4(v, v, v, v);
            for (uint64_t i = tid; i < n4; i += stride) ((uint4*)p)[i] = w;
            head = n4 * 4;
        }
        for (uint64_t i = head + tid; i < n; i += stride) p[i] = v;
    }
}

// ---------------------------------------------------------------------------
// exclusive scan: tile of SCAN_T threads x SCAN_ITEMS items
// ---------------------------------------------------------------------------
constexpr int SCAN_T = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_T * SCAN_ITEMS;

__device__ __forceinline__ uint64_t scan_item(ScanKind kind, const void* in, size_t i) {
    switch (kind) {
    case SCAN_WORDS_P: return cdiv32(((const PairDesc*)in)[i].p_len);
    case SCAN_WORDS_T: return cdiv32(((const PairDesc*)in)[i].t_len);
    case SCAN_WORDS_LEN: return cdiv32(((const uint32_t*)in)[i]);
    default: return ((const uint32_t*)in)[i];
    }
}

// inclusive scan of one value per thread over the block; returns the block total
__device__ uint64_t block_inclusive_scan(uint64_t& v) {
    __shared__ uint64_t wsum[SCAN_T / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 1; off < 64; off <<= 1) {
        uint64_t u = __shfl_up(v, off);
        if (lane >= off) v += u;
    }
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
    uint64_t before = 0, total = 0;
    for (int w = 0; w < SCAN_T / 64; w++) {
        if (w < wave) before += wsum[w];
        total += wsum[w];
    }
    v += before;
    __syncthreads();
    return total;
}

// Two passes over tiles of SCAN_TILE items.  Thread t of a tile takes items
// t, t + SCAN_T, ... (each load and store of a wavefront is one contiguous
// run); the first pass writes each tile's total, the second scans the tile
// in SCAN_ITEMS block-wide rounds on top of the totals of the tiles before
// it, which every block sums for itself.
__global__ __launch_bounds__(SCAN_T) void k_scan_partial(ScanKind kind, const void* in, size_t n,
                                                         uint64_t* block_sums) {
    const size_t base = (size_t)blockIdx.x * SCAN_TILE + threadIdx.x;
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        const size_t i = base + (size_t)j * SCAN_T;
        if (i < n) s += scan_item(kind, in, i);
    }
    const uint64_t total = block_inclusive_scan(s);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Up to SCAN_SELF_MAX tiles each block of the second pass sums the totals of
// the tiles before it itself; beyond, a one-block pass turns the totals into
// exclusive prefixes first (the sums would grow with the square of the tiles).
constexpr size_t SCAN_SELF_MAX = 8192;

__global__ __launch_bounds__(SCAN_T) void k_scan_blocks(uint64_t* block_sums, size_t nb) {
    uint64_t carry = 0;
    for (size_t base = 0; base < nb; base += SCAN_T) {
        const size_t i = base + threadIdx.x;
        uint64_t v = i < nb ? block_sums[i] : 0;
        const uint64_t mine = v;
        const uint64_t total = block_inclusive_scan(v);
        if (i < nb) block_sums[i] = carry + v - mine;  // exclusive
        carry += total;
    }
}

__global__ __launch_bounds__(SCAN_T) void k_scan_final(ScanKind kind, const void* in, size_t n,
                                                       const uint64_t* block_sums, int prefixed,
                                                       uint64_t* out) {
    uint64_t carry;
    if (prefixed) {
        carry = block_sums[blockIdx.x];
    } else {
        uint64_t before = 0;
        for (size_t b = threadIdx.x; b < blockIdx.x; b += SCAN_T) before += block_sums[b];
        carry = block_inclusive_scan(before);  // the block total: tiles before this one
    }
    const size_t base = (size_t)blockIdx.x * SCAN_TILE + threadIdx.x;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        const size_t i = base + (size_t)j * SCAN_T;
        const uint64_t v = i < n ? scan_item(kind, in, i) : 0;
        uint64_t incl = v;
        const uint64_t total = block_inclusive_scan(incl);
        if (i < n) out[i] = carry + incl - v;
        carry += total;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = carry;
}

// A short scan (the bucket histogram): one block walks the tiles in order,
// carrying the running total, and writes the total to out[n].
constexpr size_t SCAN_SINGLE_MAX = 8 * (size_t)SCAN_TILE;
__global__ __launch_bounds__(SCAN_T) void k_scan_single(ScanKind kind, const void* in, size_t n,
                                                        uint64_t* out) {
    uint64_t carry = 0;
    for (size_t tile = 0; tile < n; tile += SCAN_TILE) {
        const size_t base = tile + (size_t)threadIdx.x * SCAN_ITEMS;
        uint64_t vals[SCAN_ITEMS];
        uint64_t s = 0;
        for (int j = 0; j < SCAN_ITEMS; j++) {
            vals[j] = base + j < n ? scan_item(kind, in, base + j) : 0;
            s += vals[j];
        }
        uint64_t incl = s;
        const uint64_t total = block_inclusive_scan(incl);
        uint64_t run = carry + incl - s;
        for (int j = 0; j < SCAN_ITEMS; j++) {
            if (base + j < n) out[base + j] = run;
            run += vals[j];
        }
        carry += total;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

// ---------------------------------------------------------------------------
// ASCII -> 2-bit packing.  One thread per output word (32 bases).
// ---------------------------------------------------------------------------
// Codes of the 4 bytes of x (A/a=0, C/c=1, G/g=2, T/t=3) in 8 bits; `bad`
// collects the bits of bytes (among the low `keep` mask) that are not one of
// those letters.  The code of an ASCII letter is bits 1-2 of the byte folded
// ((c >> 1) ^ (c >> 2)) & 3; a byte is valid when the lowercase letter of its
// code (looked up bytewise with v_perm_b32) equals the byte in lowercase.
__device__ __forceinline__ uint32_t pack4(uint32_t x, uint32_t keep, uint32_t& bad) {
    const uint32_t c = ((x >> 1) ^ (x >> 2)) & 0x03030303u;
    // bytes 'a' 'c' 'g' 't' selected by c (selector values 0..3 pick bytes of src1)
    const uint32_t letters = __builtin_amdgcn_perm(0u, 0x74676361u, c);
    bad |= (letters ^ (x | 0x20202020u)) & keep;
    uint32_t v = c & keep;
    v = (v | (v >> 6)) & 0x000F000Fu;
    return (v | (v >> 12)) & 0xFFu;
}

// 32 bases starting at byte b0 of `ascii` (cnt of them valid, 1..32) as one
// 2-bit word.  Reads the aligned dwords covering the bases; near the end of
// the sequence the dword index is clamped to the last one holding a base,
// so no byte past the sequence is read.
__device__ __forceinline__ uint64_t pack_word(const uint8_t* __restrict__ ascii, uint64_t b0,
                                              int cnt, bool& ok) {
    const uint8_t* first = ascii + b0;
    const uint32_t sh = (uint32_t)((uintptr_t)first & 3u);
    const uint32_t* src = (const uint32_t*)(first - sh);
    const int lastd = (int)((sh + cnt - 1) >> 2);  // last dword holding a base
    uint32_t raw[9];
    if (lastd == 8) {
#pragma unroll
        for (int d = 0; d < 9; d++) raw[d] = src[d];
    } else {
#pragma unroll
        for (int d = 0; d < 9; d++) raw[d] = src[min(d, lastd)];
    }
    uint64_t word = 0;
    uint32_t bad = 0;
#pragma unroll
    for (int d = 0; d < 8; d++) {
        const uint32_t x = __builtin_amdgcn_alignbyte(raw[d + 1], raw[d], sh);
        const int c = min(max(cnt - 4 * d, 0), 4);
        const uint32_t keep = c >= 4 ? 0xFFFFFFFFu : ((1u << (8 * c)) - 1u);
        word |= (uint64_t)pack4(x, keep, bad) << (8 * d);
    }
    ok = bad == 0;
    return word;
}

// blockIdx.y selects the side: 0 patterns, 1 texts
__global__ void k_pack_pairs(const PairDesc* __restrict__ pairs, size_t n,
                             const uint8_t* __restrict__ pascii, const uint8_t* __restrict__ tascii,
                             const uint64_t* __restrict__ ws_p, const uint64_t* __restrict__ ws_t,
                             uint32_t max_words_p, uint32_t max_words_t,
                             uint64_t* __restrict__ words_p, uint64_t* __restrict__ words_t,
                             PairDesc* __restrict__ packed, unsigned long long* err_pair) {
    const int which = blockIdx.y;
    const uint8_t* ascii = which ? tascii : pascii;
    const uint64_t* word_starts = which ? ws_t : ws_p;
    const uint32_t max_words = which ? max_words_t : max_words_p;
    uint64_t* words = which ? words_t : words_p;
    const size_t total = n * (size_t)max_words;
    const bool narrow = total <= 0xFFFFFFFFull;  // 32-bit division suffices
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        const size_t i = narrow ? (size_t)((uint32_t)t / max_words) : t / max_words;
        const uint32_t w = (uint32_t)(t - i * max_words);
        const PairDesc d = pairs[i];
        const uint32_t len = which ? d.t_len : d.p_len;
        const uint64_t start = which ? d.t_start : d.p_start;
        // word starts: a scan, or (no scan) a fixed stride of max_words
        const uint64_t ws = word_starts ? word_starts[i] : (uint64_t)i * max_words;
        if (w == 0) {
            if (which) {
                packed[i].t_start = ws;
                packed[i].t_len = d.t_len;
            } else {
                packed[i].p_start = ws;
                packed[i].p_len = d.p_len;
            }
        }
        const uint32_t nw = cdiv32(len);
        if (w >= nw) continue;
        int cnt = (int)min(32u, len - 32u * w);
        bool ok = true;
        words[ws + w] = pack_word(ascii, start + 32ull * w, cnt, ok);
        if (!ok) atomicMin(err_pair, (unsigned long long)i);
    }
}

__global__ void k_pack_seqs(const uint8_t* __restrict__ ascii, const uint64_t* __restrict__ starts,
                            const uint32_t* __restrict__ lens, size_t n,
                            const uint64_t* __restrict__ word_starts, uint64_t total_words,
                            uint64_t* __restrict__ words, unsigned long long* err_index) {
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < total_words;
         t += (uint64_t)gridDim.x * blockDim.x) {
        // sequence holding word t: the last i with word_starts[i] <= t.  Start
        // from the guess of equal lengths and widen by doubling steps until
        // the bracket holds t, then bisect (exact at once for equal lengths).
        size_t g = (size_t)((double)t * (double)n / (double)total_words);
        g = g < n ? g : n - 1;
        size_t lo, hi;  // invariant: word_starts[lo] <= t < word_starts[hi] (hi = n: end)
        if (word_starts[g] <= t) {
            lo = g;
            size_t step = 1;
            hi = g + 1;
            while (hi < n && word_starts[hi] <= t) {
                lo = hi;
                hi = hi + step < n ? hi + step : n;
                step <<= 1;
            }
        } else {
            hi = g;
            size_t step = 1;
            lo = g >= 1 ? g - 1 : 0;
            while (lo > 0 && word_starts[lo] > t) {
                hi = lo;
                lo = lo >= step ? lo - step : 0;
                step <<= 1;
            }
        }
        while (hi - lo > 1) {
            const size_t mid = (lo + hi) >> 1;
            if (word_starts[mid] <= t) lo = mid; else hi = mid;
        }
        const size_t i = lo;
        const uint32_t w = (uint32_t)(t - word_starts[i]);
        const uint32_t len = lens[i];
        int cnt = (int)min(32u, len - 32u * w);
        bool ok = true;
        words[t] = pack_word(ascii, starts[i] + 32ull * w, cnt, ok);
        if (!ok) atomicMin(err_index, (unsigned long long)i);
    }
}

// ---------------------------------------------------------------------------
// Short-pair kernel.
//
// A lane group of G lanes aligns one pair; 64/G groups share a wave and step
// through scores together.  The group holds a window of W = G*DPL diagonals
// kmin .. kmin+W-1, centred between diagonal 0 and the target diagonal m-n,
// as DPL layers of G diagonals: layer 0 is the middle G, each further layer
// adds G/2 diagonals on each side.  A layer is computed only once the
// wavefront has reached the edge of the layer inside it -- until then every
// cell in it is NULL -- and a wave skips the layers none of its groups needs,
// so early (narrow) score steps cost one layer.
//
// LDS per lane group.  Row r of an offset store holds, for one score step,
// the offsets of the W diagonals plus a NULL pad on each side, so
// neighbouring diagonals are read without bounds checks.  I and D rows form
// rings of e + 1 steps (a step reads them back e steps).  M rows form a ring
// of max(x, o + e) + 1 steps in score mode; in CIGAR mode every M row of the
// pair is kept (steps 0..cap after one NULL row, which stands for every step
// before 0), and each cell of
// each step gets a 4-bit decision record (two cells per byte): the source of
// M before extension (mismatch, end of insertion, end of deletion) and
// whether I and D opened from M.  Every row starts NULL.  Offsets are int8
// when both sequences are shorter than 128 bases (twice the lane groups per
// CU), int16 otherwise.
//
// A pair leaves the kernel through the overflow list (and is finished by the
// general kernel) when its wavefront touches a window edge before reaching
// the end, when it needs more than `cap` steps, when a sequence does not fit
// the LDS words, or when its runs overflow the slot.  Values are never
// computed from an incomplete window.
// ---------------------------------------------------------------------------

// Whether any lane of the caller's lane group (64/G groups per wave) has its
// bit set in the wave-wide ballot `b`.
template <int G>
__device__ __forceinline__ bool group_any(uint64_t b, int gshift) {
    constexpr uint64_t GMASK = G == 64 ? ~0ULL : ((1ULL << G) - 1ULL);
    return ((b >> gshift) & GMASK) != 0;
}

// Window index of lane l's diagonal in layer d (see above).
template <int G, int DPL>
__device__ __forceinline__ int layer_index(int l, int d) {
    constexpr int W = G * DPL;
    if (DPL == 1) return l;
    if (d == 0) return W / 2 - G / 2 + l;
    return l < G / 2 ? W / 2 - G / 2 - d * (G / 2) + l : W / 2 + G / 2 + (d - 1) * (G / 2) + (l - G / 2);
}

template <class RowT>
struct RowNull;
template <>
struct RowNull<int8_t> {
    static constexpr int value = -128;
};
template <>
struct RowNull<int16_t> {
    static constexpr int value = -16384;
};

template <int G, int DPL, bool CIGAR, class RowT, bool ENDS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_short(
    ShortArgs a, int persistent) {
    extern __shared__ __align__(16) unsigned char lds[];
    constexpr int W = G * DPL;
    constexpr int RW = W + 2;
    constexpr int GPW = 64 / G;
    // NULL; it drifts up by at most one per step and stays negative
    constexpr int NUL = RowNull<RowT>::value;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const int grp = lane / G;
    const int gl = lane - grp * G;
    const int gshift = grp * G;

    lds_ptr<unsigned char> gbase = (lds_ptr<unsigned char>)lds + (wave * GPW + grp) * a.group_bytes;
    lds_ptr<RowT> RM = (lds_ptr<RowT>)gbase;
    lds_ptr<RowT> RI = (lds_ptr<RowT>)(gbase + a.id_off);
    lds_ptr<RowT> RD = RI + a.ring2 * RW;
    const int rows_bytes = a.rows_bytes;
    // CIGAR mode: 4-bit decision records of steps 0..cap, two cells per byte
    // (cell j in the low nibble when j is even): bits 0-1 the source of M
    // (0 mismatch, 1 end of insertion, 2 end of deletion), bit 2 insertion
    // opened from M, bit 3 deletion opened from M
    lds_ptr<uint8_t> FL = (lds_ptr<uint8_t>)(gbase + rows_bytes);
    const int rec_bytes = CIGAR ? (((a.cap + 1) * (W / 2)) + 15) & ~15 : 0;
    // CIGAR mode: the backtrace stages its runs over the I/D rings (free by then)
    lds_ptr<uint32_t> STAGE = (lds_ptr<uint32_t>)(gbase + a.id_off);
    lds_ptr<uint64_t> SP64 = (lds_ptr<uint64_t>)(gbase + rows_bytes + rec_bytes);
    lds_ptr<uint64_t> ST64 = SP64 + a.seq_words;
    lds_ptr<const uint32_t> SP = (lds_ptr<const uint32_t>)SP64;
    lds_ptr<const uint32_t> ST = (lds_ptr<const uint32_t>)ST64;

    const int X = a.pen.x, OE = a.pen.oe, E = a.pen.e, PRE = a.pen.pre;
    const int ring = a.ring, ring2 = a.ring2;

    const bool bnd = gl == 0 || gl == G - 1;  // lanes on a layer's outermost diagonals
    int jl[DPL];  // window index of each of this lane's diagonals
#pragma unroll
    for (int d = 0; d < DPL; d++) jl[d] = layer_index<G, DPL>(gl, d);

    // persistent: a wave claims `queue_chunk` rounds of GPW queue entries per
    // atomic and works through them before claiming again.  The runs of the
    // pairs of a claim go, packed, into the claim's share of the slots
    // (slot_cap words per entry): `wbump` is the next free word.
    uint32_t claim = 0, claim_left = 0;
    uint64_t wbump = 0;
    for (uint32_t iter = 0;; iter++) {
        uint32_t qbase;
        if (persistent) {
            if (claim_left == 0) {
                uint32_t t = 0;
                if (lane == 0) t = atomicAdd(a.queue, (uint32_t)(GPW * a.queue_chunk));
                claim = __builtin_amdgcn_readfirstlane(t);
                claim_left = (uint32_t)a.queue_chunk;
                wbump = (uint64_t)claim * a.slot_cap;
            }
            qbase = claim;
            claim += GPW;
            claim_left--;
        } else {
            if (iter) break;
            qbase = (blockIdx.x * wpb + wave) * GPW;
            wbump = (uint64_t)qbase * a.slot_cap;
        }
        if (qbase >= a.num) break;
        const uint32_t q = qbase + grp;
        uint32_t pair = 0;
        int n = 0, m = 0;
        uint64_t ps = 0, ts = 0;
        bool active_ok = q < a.num;
        if (active_ok) {
            pair = a.order ? a.order[q] : q;
            if (pair >= a.npairs) {  // a corrupt permutation must not fault: skip the entry
                active_ok = false;
                pair = 0;
            }
        }
        if (active_ok) {
            const PairDesc d = a.pairs[pair];
            n = (int)d.p_len;
            m = (int)d.t_len;
            ps = d.p_start;
            ts = d.t_start;
        }
        const int kt = m - n;
        const int kmin = (kt >> 1) - W / 2;
        const int nwp = (n + 31) >> 5, nwt = (m + 31) >> 5;
        // ends-free: the pair's free ends (the start diagonals -pbc .. tbc)
        const int pbc = ENDS ? min(a.ends.pb, n) : 0, pec = ENDS ? min(a.ends.pe, n) : 0;
        const int tbc = ENDS ? min(a.ends.tb, m) : 0, tec = ENDS ? min(a.ends.te, m) : 0;
        // 0 running, 1 finished or idle, 2 overflow
        int st = active_ok ? 0 : 1;
        const bool fits = ENDS ? (kmin <= -pbc && tbc < kmin + W)
                               : (kmin <= 0 && 0 < kmin + W && kmin <= kt && kt < kmin + W);
        if (active_ok && !(fits && nwp + 1 <= a.seq_words && nwt + 1 <= a.seq_words)) st = 2;

        // stage both sequences (zero past their ends)
        for (int w = gl; w < a.seq_words; w += G) {
            SP64[w] = (st == 0 && w < nwp) ? a.pw[ps + w] : 0ULL;
            ST64[w] = (st == 0 && w < nwt) ? a.tw[ts + w] : 0ULL;
        }
        // every offset row starts NULL (pads included); the M rows and the
        // I/D rings are contiguous and padded to 16 bytes
        {
            constexpr uint32_t NW = sizeof(RowT) == 1 ? 0x80808080u : 0xC000C000u;
            static_assert(sizeof(RowT) == 1 ? (int8_t)0x80 == NUL : (int16_t)0xC000 == NUL,
                          "fill word must repeat NULL");
            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
            lds_ptr<u32x4> f = (lds_ptr<u32x4>)gbase;
            for (int idx = gl; idx < rows_bytes / 16; idx += G) f[idx] = u32x4{NW, NW, NW, NW};
        }
        wave_sync();

        // per diagonal: the largest admissible offset min(m, n + k) (negative
        // off the matrix), the same floored at 0, and the diagonal itself
        int lim[DPL], limz[DPL], kd[DPL];
#pragma unroll
        for (int d = 0; d < DPL; d++) {
            kd[d] = kmin + jl[d];
            lim[d] = min(m, n + kd[d]);
            limz[d] = max(lim[d], 0);
        }
        const int jt = kt - kmin;  // window index of the target diagonal
        int S = 0;
        // layers this group computes: at first the fewest that hold diagonal 0
        int lay = 1;
        {
            const int j0 = -pbc - kmin, j1 = tbc - kmin;  // the start diagonals
            while (lay < DPL && (j0 < W / 2 - G / 2 - (lay - 1) * (G / 2) ||
                                 j1 > W / 2 + G / 2 - 1 + (lay - 1) * (G / 2)))
                lay++;
        }
        int endj = W;  // ends-free CIGAR: lowest window index of an end cell
        // Offsets (in cells, + 1 for the pad) of the current M and I/D rows,
        // kept as running sums (scalar adds, no multiplies): M row of step 0
        // after the NULL rows, I/D row of step 0 last in its ring.
        const int RINGM = ring * RW, RINGID = ring2 * RW;
        const int XRW = X * RW, OERW = OE * RW, ERW = E * RW;
        int ocur = (CIGAR ? 1 : PRE) * RW + 1;
        int ocur2 = (ring2 - 1) * RW + 1;
        for (int s = 0;; s++) {
            if (__ballot(st == 0) == 0) break;
            // layers the wave computes this step: the most any of its groups needs
            int nlay = 1;
#pragma unroll
            for (int d = 1; d < DPL; d++) nlay += __ballot(st == 0 && lay > d) != 0 ? 1 : 0;
            const bool growable = DPL > 1 && __ballot(st == 0 && lay < DPL) != 0;
            if (s > 0) {
                ocur += RW;  // never wraps in CIGAR mode
                ocur -= ocur > RINGM ? RINGM : 0;
                ocur2 += RW;
                ocur2 -= ocur2 > RINGID ? RINGID : 0;
            }
            int ox = ocur - XRW, oo = ocur - OERW, oe = ocur2 - ERW;
            if (CIGAR) {  // steps before 0 read the NULL row
                ox = max(ox, 1);
                oo = max(oo, 1);
            } else {
                ox += ox < 1 ? RINGM : 0;
                oo += oo < 1 ? RINGM : 0;
            }
            oe += oe < 1 ? RINGID : 0;
            lds_ptr<const RowT> mx = RM + ox;
            lds_ptr<const RowT> mo = RM + oo;
            lds_ptr<const RowT> il = RI + oe;
            lds_ptr<const RowT> dr = RD + oe;
            const bool run = st == 0;
            // Layers one after another (cells of a step read only earlier
            // steps' rows, so the order does not matter): compute the cells,
            // extend them, store the row and the decision records, and note
            // termination, window-edge and layer-growth conditions.
            bool term = false, edge = false, grow = false;
            int tj = W;  // lowest window index of this lane's end cells this step
#pragma unroll
            for (int d = 0; d < DPL; d++) {
                if (d >= nlay) break;
                const int j = jl[d];
                const int L = lim[d];
                int Mv, Iv = NUL, Dv = NUL, rec = 0;
                if (s == 0) {
                    if (ENDS)  // the free starts: M_0[k] = max(k, 0) for -pbc <= k <= tbc
                        Mv = (kd[d] >= -pbc && kd[d] <= tbc) ? max(kd[d], 0) : NUL;
                    else
                        Mv = (kmin + j == 0) ? 0 : NUL;
                } else {
                    // Candidates as distances t = L - c below the diagonal's limit
                    // L: an admissible offset has 0 <= t <= L, a NULL source
                    // (negative, drifting up by at most one per step) has
                    // L < t <= L - NUL, and an offset past L has t < 0, which
                    // is huge as unsigned.  So the largest admissible candidate
                    // is the unsigned minimum, floored at NULL (t = L - NUL),
                    // and over-long candidates are dropped before the maximum.
                    const uint32_t tn = (uint32_t)(L - NUL);
                    const uint32_t ta = (uint32_t)(L - 1 - mo[j - 1]);  // open from M
                    const uint32_t tb = (uint32_t)(L - 1 - il[j - 1]);  // extend I
                    const uint32_t tc = (uint32_t)(L - mo[j + 1]);      // open from M
                    const uint32_t te = (uint32_t)(L - dr[j + 1]);      // extend D
                    const uint32_t tx = (uint32_t)(L - 1 - mx[j]);      // mismatch
                    const uint32_t ti = min(min(ta, tb), tn);
                    const uint32_t td = min(min(tc, te), tn);
                    const uint32_t tm = min(min(tx, ti), td);
                    Mv = L - (int)tm;
                    Iv = L - (int)ti;
                    Dv = L - (int)td;
                    if (CIGAR) {
                        // decisions the backtrace replays (tie-break: mismatch,
                        // then insertion, then deletion; gap open before extend)
                        const int msrc = tx == tm ? 0 : (ti == tm ? 1 : 2);
                        rec = msrc | (ta == ti ? 4 : 0) | (tc == td ? 8 : 0);
                    }
                }
                // Extend along matches, 32 bases per compare.  The loop is
                // wave-uniform: while any lane extends, every lane runs the
                // compare, lanes that do not extend at offset 0 (in bounds)
                // with nothing left (rem: bases before either sequence ends,
                // min(n - v, m - h) = L - h).
                {
                    const bool go = run && (unsigned)Mv < (unsigned)limz[d];
                    int hp = go ? Mv : 0;
                    int vp = go ? Mv - kd[d] : 0;
                    int rem = go ? limz[d] - Mv : 0;
                    uint64_t gm = __ballot(go);
                    while (gm) {
                        const int r = min(common_prefix(window32(SP, vp), window32(ST, hp)), rem);
                        hp += r;
                        vp += r;
                        rem = r == 32 ? rem - 32 : 0;
                        gm = __ballot(rem > 0);
                    }
                    Mv = go ? hp : Mv;
                }
                // store the step's row (groups that stopped write rows nobody reads)
                RM[ocur + j] = (RowT)Mv;
                RI[ocur2 + j] = (RowT)Iv;
                RD[ocur2 + j] = (RowT)Dv;
                if (CIGAR) {
                    // neighbouring lanes hold neighbouring diagonals (even j on
                    // even lanes): both write the byte of the pair of cells
                    const int other = __builtin_amdgcn_update_dpp(0, rec, 0xB1, 0xF, 0xF, false);
                    const int lo = (gl & 1) ? other : rec;
                    const int hi = (gl & 1) ? rec : other;
                    FL[(s * W + j) >> 1] = (uint8_t)(lo | (hi << 4));  // s <= cap here
                }
                const bool live = Mv >= 0;  // M is at least I and D
                if (ENDS) {
                    // an end cell: the last text column with at most pec
                    // pattern bases left, or the last pattern row with at
                    // most tec text bases left
                    const int vv = Mv - kd[d];
                    const bool tc = live && ((Mv == m && vv >= n - pec) || (vv == n && Mv >= m - tec));
                    term |= tc;
                    if (CIGAR) tj = tc ? min(tj, j) : tj;
                } else {
                    term |= (j == jt) & (Mv == m);
                }
                if (d == DPL - 1) edge |= bnd & live;
                if (d < DPL - 1) grow |= (d == lay - 1) & bnd & live;
            }
            const bool gterm = group_any<G>(__ballot(term), gshift);
            // the outermost layer can only be live once it is computed, and a
            // layer is only added while some running group has one to add
            bool gedge = false, ggrow = false;
            if (nlay == DPL) gedge = group_any<G>(__ballot(edge), gshift);
            if (DPL > 1 && growable) ggrow = group_any<G>(__ballot(grow), gshift);
            S = (run && gterm) ? s : S;
            if (ENDS && CIGAR) endj = (run && gterm) ? tj : endj;
            st = run ? (gterm ? 1 : ((gedge || s >= a.cap) ? 2 : 0)) : st;
            lay += (run && ggrow) ? 1 : 0;
            wave_sync();
        }

        // ends-free CIGAR: the end cell on the group's lowest diagonal
        if (ENDS && CIGAR) {
#pragma unroll
            for (int off = G / 2; off >= 1; off >>= 1) endj = min(endj, __shfl_xor(endj, off));
        }
        // results: the group leader walks the backtrace
        int cnt = 0;  // runs the group copies out (CIGAR, pair finished here)
        if (active_ok && gl == 0) {
            bool overflow = st == 2;
            if (!overflow && CIGAR) {
                const int cap_runs = a.slot_cap;
                int nr = 0, cop = -1, clen = 0;
                int s = S, k = kt, h = m;  // an M cell and its offset after extension
                if (ENDS) {
                    const int je = min(endj, W - 1);
                    k = kmin + je;
                    h = RM[(S + 1) * RW + 1 + je];
                    // the free suffix opens the run list (runs are last to first)
                    if (n - (h - k) > 0) {
                        cop = OP_D;
                        clen = n - (h - k);
                    } else if (m - h > 0) {
                        cop = OP_I;
                        clen = m - h;
                    }
                }
                // Replays the decisions recorded in the forward pass, one event
                // per iteration: at M cell (s, k) it finds where M came from
                // (a mismatch from M at s - x, or the end of a gap whose chain
                // of I or D cells it follows back to where the gap opened from
                // an M cell), emits the cell's match run (its offset minus the
                // offset before extension, which the source gives) and the
                // event's edit run, and moves to the source M cell.  An edit
                // run extends the open run when nothing matched in between and
                // the op is the same.  Both candidate runs are stored every
                // iteration at the next free stage word and only kept (the
                // count advanced) when real; stores of a walk past the stage's
                // end land on its two spare words, and the pair is then re-run
                // elsewhere.  Every iteration lowers s, so the walk ends.
                for (;;) {
                    const int j = k - kmin;
                    if (s < 0 || (unsigned)j >= (unsigned)W) {
                        overflow = true;  // inconsistent walk: leave it to the general kernel
                        break;
                    }
                    int h0 = 0, hn = 0, L = 1, op = OP_M, s2 = 0, dk = 0;
                    if (s > 0) {
                        const int f = (FL[(s * W + j) >> 1] >> ((j & 1) << 2)) & 15;
                        const int ms = f & 3;
                        if (ms == 0) {
                            hn = RM[max(s - X + 1, 0) * RW + 1 + j];
                            h0 = hn + 1;
                            s2 = s - X;
                        } else {
                            const int bit = ms == 1 ? 4 : 8;
                            const int dj = ms == 1 ? -1 : 1;
                            int sc = s, jc = j, fc = f;
                            while (!(fc & bit)) {  // still extending: one step back
                                sc -= E;
                                jc += dj;
                                if (sc <= 0 || (unsigned)jc >= (unsigned)W) break;
                                L++;
                                fc = (FL[(sc * W + jc) >> 1] >> ((jc & 1) << 2)) & 15;
                            }
                            if (!(fc & bit)) {
                                overflow = true;  // a gap with no opening: inconsistent
                                break;
                            }
                            hn = RM[max(sc - OE + 1, 0) * RW + 1 + jc + dj];
                            h0 = ms == 1 ? hn + L : hn;  // insertions consume text
                            s2 = sc - OE;
                            dk = dj * L;
                        }
                        op = ms + 1;  // op codes: X=1 I=2 D=3
                    }
                    const bool last = s == 0;
                    // ends-free: M_0[k] = max(k, 0) before extension, after a
                    // free prefix of k text (k > 0) or -k pattern (k < 0) bases
                    int fop = -1, flen = 0;
                    if (ENDS && last) {
                        h0 = max(k, 0);
                        fop = k > 0 ? OP_I : (k < 0 ? OP_D : -1);
                        flen = k > 0 ? k : -k;
                    }
                    const int mlen = h - h0;
                    if (mlen < 0 || hn < 0) {
                        overflow = true;
                        break;
                    }
                    const bool hasM = mlen > 0;
                    if (ENDS && !hasM && fop >= 0 && cop == fop) {  // one run with the prefix
                        clen += flen;
                        fop = -1;
                    }
                    const bool flush = cop >= 0 && (hasM || last || cop != op);
                    STAGE[min(nr, cap_runs + 1)] = ((uint32_t)clen << 4) | (uint32_t)cop;
                    nr += flush ? 1 : 0;
                    STAGE[min(nr, cap_runs + 1)] = ((uint32_t)mlen << 4) | (uint32_t)OP_M;
                    nr += hasM ? 1 : 0;
                    if (ENDS && fop >= 0) {
                        STAGE[min(nr, cap_runs + 1)] = ((uint32_t)flen << 4) | (uint32_t)fop;
                        nr++;
                    }
                    if (last) break;
                    clen = (flush || hasM) ? L : clen + L;
                    cop = op;
                    s = s2;
                    k += dk;
                    h = hn;
                }
                if (overflow || nr > cap_runs) overflow = true;
                else cnt = nr;
            }
            if (overflow) {
                const uint32_t at = atomicAdd(a.ovf_count, 1u);
                a.ovf_list[at] = pair;
            } else {
                a.scores[pair] = S * a.pen.g;
                if (!CIGAR) a.nruns[pair] = 0;
            }
            if (CIGAR && !overflow) cnt = max(cnt, 0) | (1 << 30);  // mark: finished here
        }
        if (CIGAR) {
            // copy the groups' staged runs out, packed one after another
            wave_sync();
            const bool done = (cnt >> 30) & 1;
            cnt &= (1 << 30) - 1;
            int pre = 0, tot = 0;
#pragma unroll
            for (int g2 = 0; g2 < GPW; g2++) {
                const int cg = __shfl(cnt, g2 * G);
                pre += g2 < grp ? cg : 0;
                tot += cg;
            }
            const int mine = __shfl(cnt, gshift);
            const uint64_t base = wbump + (uint64_t)pre;
            for (int r = gl; r < mine; r += G) a.slots[base + r] = STAGE[r];
            if (done) {
                a.nruns[pair] = (uint32_t)cnt;
                a.run_src[pair] = base + a.run_src_add;
            }
            wbump += (uint64_t)tot;
        }
        wave_sync();
    }
}

// ---------------------------------------------------------------------------
// General kernel: one workgroup per pair, any length, any score.
//
// Slice layout (bytes): a ring of pre + 1 full-width slots of M, I and D
// rows (int32, diagonals [-n - 1, m + 1]) that the score steps work in, and
// a slot of NULL rows.  CIGAR mode adds, after the ring, one history row per
// step that grows towards the end of the slice: the step's M offsets (16-bit
// while the text is shorter than 65535 bases, else 32-bit) and a 4-bit
// decision record per diagonal (as in the short kernel); the step table
// {lo, hi, offset} grows down from the end, and the backtrace writes
// reversed runs into the gap.
// ---------------------------------------------------------------------------
struct RowMeta {
    int lo, hi;
    long long off;  // byte offset of the row in the slice; -1: no wavefront
};

template <bool SEQ_LDS>
struct SeqView {
    const uint32_t* p;
    const uint32_t* t;
    int np32, nt32;  // valid dwords (global variant bounds reads)
    __device__ __forceinline__ uint32_t P(int q) const {
        if (SEQ_LDS) return p[q];
        return q < np32 ? p[q] : 0u;
    }
    __device__ __forceinline__ uint32_t T(int q) const {
        if (SEQ_LDS) return t[q];
        return q < nt32 ? t[q] : 0u;
    }
    // 16 bases from base `pos` on (one 32-bit funnel shift)
    __device__ __forceinline__ uint32_t win16P(int pos) const {
        const int q = pos >> 4;
        return __builtin_amdgcn_alignbit(P(q + 1), P(q), (uint32_t)(pos & 15) << 1);
    }
    __device__ __forceinline__ uint32_t win16T(int pos) const {
        const int q = pos >> 4;
        return __builtin_amdgcn_alignbit(T(q + 1), T(q), (uint32_t)(pos & 15) << 1);
    }
    __device__ __forceinline__ uint64_t winP(int pos) const {
        const int q = pos >> 4;
        const uint32_t b = (uint32_t)(pos & 15) << 1;
        const uint32_t w0 = P(q), w1 = P(q + 1), w2 = P(q + 2);
        return ((uint64_t)__builtin_amdgcn_alignbit(w2, w1, b) << 32) |
               __builtin_amdgcn_alignbit(w1, w0, b);
    }
    __device__ __forceinline__ uint64_t winT(int pos) const {
        const int q = pos >> 4;
        const uint32_t b = (uint32_t)(pos & 15) << 1;
        const uint32_t w0 = T(q), w1 = T(q + 1), w2 = T(q + 2);
        return ((uint64_t)__builtin_amdgcn_alignbit(w2, w1, b) << 32) |
               __builtin_amdgcn_alignbit(w1, w0, b);
    }
};

template <bool SEQ_LDS>
__device__ __forceinline__ int extend_general(const SeqView<SEQ_LDS>& sv, int n, int m, int k,
                                              int h) {
    int v = h - k;
    // a 16-base compare first: most cells of a long, divergent pair stop
    // within it, and a wave runs on to the 32-base compares only while one
    // of its lanes still matches
    if (v < n && h < m) {
        const uint32_t d = sv.win16P(v) ^ sv.win16T(h);
        int r = d ? (int)(__builtin_ctz(d) >> 1) : 16;
        r = min(r, min(n - v, m - h));
        v += r;
        h += r;
        if (r < 16) return h;
    }
    while (v < n && h < m) {
        int r = common_prefix(sv.winP(v), sv.winT(h));
        r = min(r, min(n - v, m - h));
        v += r;
        h += r;
        if (r < 32) break;
    }
    return h;
}

// One cell of step s > 0 on diagonal k from its five source offsets: va = M
// of s - o - e and vb = I of s - e on k - 1 (insertion), vc = M of s - o - e
// and ve = D of s - e on k + 1 (deletion), vx = M of s - x on k (mismatch).
// Candidates are compared as unsigned distances t = L - c below the
// diagonal's limit L = min(m, n + k): admissible offsets 0 <= t <= L, NULL
// sources L < t <= L - NULL, offsets past L negative (huge); the maximum
// admissible candidate is the minimum t, floored at NULL.  Returns M before
// extension, I and D (negative: NULL) and the decision record the backtrace
// replays (tie-break: mismatch, then insertion, then deletion; gap open
// before extend).
struct GenCell {
    int m, i, d, rec;
};

__device__ __forceinline__ GenCell general_cell(int n, int m, int k, int va, int vb, int vc, int ve,
                                                int vx) {
    const int L = min(m, n + k);
    const uint32_t tn = (uint32_t)(L - NUL32);
    const uint32_t ta = (uint32_t)(L - 1 - va);
    const uint32_t tb = (uint32_t)(L - 1 - vb);
    const uint32_t tc = (uint32_t)(L - vc);
    const uint32_t te = (uint32_t)(L - ve);
    const uint32_t tx = (uint32_t)(L - 1 - vx);
    const uint32_t ti = min(min(ta, tb), tn);
    const uint32_t td = min(min(tc, te), tn);
    const uint32_t tm = min(min(tx, ti), td);
    GenCell c;
    c.m = L - (int)tm;
    c.i = L - (int)ti;
    c.d = L - (int)td;
    const int msrc = tx == tm ? 0 : (ti == tm ? 1 : 2);
    c.rec = msrc | (ta == ti ? 4 : 0) | (tc == td ? 8 : 0);
    return c;
}

// LDS bytes of the general kernel's metadata ring and slot ranges for a ring
// of R steps (16-byte aligned; the staged sequences follow)
__host__ __device__ __forceinline__ int general_meta_lds(int R) { return (R * 24 + 15) & ~15; }

// RowT: int16_t ring rows while every offset fits (texts shorter than 32767
// bases), halving the ring's memory traffic, else int32_t.  Stored NULLs are
// normalised to RNUL, so no NULL drifts up over many steps.
// Eight wavefronts per SIMD (the compiler holds the kernel to 78 SGPRs; 106
// left it at seven): more pairs resident hide more of each step's latency
// (100 k pairs of 1-10 kbp: 425 against 443 ms score-only, 564 against 581 ms
// with checkpoint CIGARs).
// HIST: the launch keeps a history row per step (CIGAR without checkpoints);
// the other forms compute no decision records.  FREE: some end is free
// (global alignment ends on the one corner cell).
template <bool SEQ_LDS, class RowT, bool HIST, bool FREE>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_general(
    GeneralArgs a) {
    constexpr int RNUL = sizeof(RowT) == 2 ? -16384 : NUL32;
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ int sh_end;  // lowest diagonal whose M cell ends the alignment
    __shared__ int sh_fail;
    __shared__ int sh_dmin, sh_klo, sh_khi;  // WF-adaptive: least distance, kept range

    const uint32_t job = blockIdx.x;
    if (job >= a.num_jobs) return;
    const uint32_t pair = a.jobs[job];
    const PairDesc desc = a.pairs[pair];
    const int n = (int)desc.p_len, m = (int)desc.t_len;
    const int tid = threadIdx.x, BT = blockDim.x;
    const int X = a.pen.x, OE = a.pen.oe, E = a.pen.e, PRE = a.pen.pre;
    const int R = PRE + 1;
    // no walk for this job unless the forward pass below succeeds
    if (a.cigar && tid == 0) a.jstate[job].S = -1;
    // dynamic LDS: the metadata ring (one entry per step of the ring), the
    // range of diagonals each ring slot holds, then (SEQ_LDS) the sequences;
    // sized to this penalty set's ring, so more workgroups fit on a CU
    RowMeta* meta = (RowMeta*)lds;
    int* wr_lo = (int*)(meta + R);
    int* wr_hi = wr_lo + R;
    unsigned char* seq_lds = lds + general_meta_lds(R);
    // free ends of this pair (global alignment: all zero)
    const int pb = min(a.ends.pb, n), pe = min(a.ends.pe, n);
    const int tb = min(a.ends.tb, m), te = min(a.ends.te, m);
    unsigned char* slice = a.arena + a.slice_off[job];
    const long long slice_bytes = (long long)(a.slice_off[job + 1] - a.slice_off[job]);

    SeqView<SEQ_LDS> sv;
    const int nwp = (n + 31) >> 5, nwt = (m + 31) >> 5;
    if (SEQ_LDS) {
        uint64_t* p64 = (uint64_t*)seq_lds;
        uint64_t* t64 = p64 + nwp + 1;
        for (int w = tid; w <= nwp; w += BT) p64[w] = w < nwp ? a.pw[desc.p_start + w] : 0ULL;
        for (int w = tid; w <= nwt; w += BT) t64[w] = w < nwt ? a.tw[desc.t_start + w] : 0ULL;
        sv.p = (const uint32_t*)p64;
        sv.t = (const uint32_t*)t64;
    } else {
        sv.p = (const uint32_t*)(a.pw + desc.p_start);
        sv.t = (const uint32_t*)(a.tw + desc.t_start);
    }
    sv.np32 = 2 * nwp;
    sv.nt32 = 2 * nwt;
    for (int r = tid; r < R; r += BT) {
        meta[r] = RowMeta{0, -1, -1};
        wr_lo[r] = 0;
        wr_hi[r] = -1;
    }
    if (tid == 0) {
        sh_end = INT_MAX;
        sh_fail = 0;
        sh_dmin = INT_MAX;
        sh_klo = INT_MAX;
        sh_khi = INT_MIN;
    }
    const int MWL = a.heur.mwl, MDT = a.heur.mdt;

    // step table (CIGAR mode) lives at the end of the slice, entry s at
    // slice_bytes - 16 * (s + 1)
    RowMeta* table = (RowMeta*)(slice + slice_bytes) - 1;
    // Ring slots of M, I and D rows indexed by diagonal: FW entries each,
    // diagonal k at k + n + 1 (one pad on each side), then one slot of NULL
    // rows that stands for steps without a wavefront.  Every slot starts
    // NULL, and a step that takes over a slot writes its range [lo, hi] and
    // NULLs whatever the slot's previous step wrote outside it, so every
    // entry outside a source step's range reads NULL and the cells read
    // their sources without range checks.
    const int FW = n + m + 3;
    // one ring slot: the M, I and D rows, padded to 16 bytes so that the
    // history and the runs after the ring stay aligned
    const long long full_row = (3LL * (long long)sizeof(RowT) * FW + 15) & ~15LL;
    // CIGAR history offsets: 16-bit (0xFFFF for NULL) while every offset
    // fits, else 32-bit
    const bool h16 = m < 0xFFFF;
    const int hbytes = h16 ? 2 : 4;
    long long bump = (R + 1) * full_row;  // CIGAR history starts after the ring
    // Checkpoint CIGAR mode (CK > 0): instead of a history row per step, the
    // ring rows of R consecutive steps are kept every CK steps, and the
    // backtrace recomputes the steps between two checkpoints, in the cone of
    // diagonals that can reach the walk's entry cell, into a segment buffer
    // of fixed size placed after the checkpoints.
    const int CK = a.cigar ? a.ckpt : 0;
    constexpr bool full_hist = HIST;  // the launcher picks HIST = cigar && CK == 0
    const int DMAX = CK ? (CK + R - 1) / E : 0;  // widest cone half-width
    const int WC = 2 * DMAX + 1;                 // cone columns
    const long long SEG_ROWB = ((long long)WC * (3 * (long long)sizeof(RowT) + 1) + 15) & ~15LL;
    const long long seg_bytes = CK ? (long long)(CK + R) * SEG_ROWB : 0;
    if (bump > slice_bytes) {
        if (tid == 0) {
            const uint32_t at = atomicAdd(a.fail_count, 1u);
            a.fail_list[at] = pair;
        }
        return;
    }
    {
        RowT* ring = (RowT*)slice;  // every slot, padding included
        const long long cnt = (R + 1) * full_row / (long long)sizeof(RowT);
        for (long long i = tid; i < cnt; i += BT) ring[i] = (RowT)RNUL;
    }
    __syncthreads();
    // a hard bound on steps: deleting all of P and inserting all of T (or a
    // lower limit the host asks for)
    long long max_score_g = (2LL * (OE - E) + (long long)(n + m) * E) + 2;
    // the heuristic may settle for a worse alignment; none costs more than
    // its n + m bases at the dearest price each
    if (MWL > 0) max_score_g = (long long)(n + m) * max(X, OE) + 2;
    if (a.step_limit > 0 && a.step_limit < max_score_g) max_score_g = a.step_limit;

    int S = -1;
    long long end_off = -1;  // ring offset of the last step's rows
    int rs = 0;  // s % R
    for (long long s = 0;; s++, rs = rs + 1 == R ? 0 : rs + 1) {
        if (s > max_score_g) {
            if (tid == 0) sh_fail = 2;
            break;
        }
        // checkpoint mode: the step table, the segment buffer and the
        // checkpoints must stay apart
        if (CK && bump + seg_bytes > slice_bytes - 16LL * (s + 2)) {
            if (tid == 0) sh_fail = 1;
            break;
        }
        // the source rows of this step (metadata ring entry of step t: t % R)
        RowMeta sx{0, -1, -1}, so{0, -1, -1}, se{0, -1, -1};
        if (s >= X) sx = meta[rs - X + (rs < X ? R : 0)];
        if (s >= OE) so = meta[rs - OE + (rs < OE ? R : 0)];
        if (s >= E) se = meta[rs - E + (rs < E ? R : 0)];
        int lo, hi;
        bool present;
        if (s == 0) {  // the free starts (diagonal 0 alone in global alignment)
            lo = -pb;
            hi = tb;
            present = true;
        } else {
            lo = 1 << 30;
            hi = -(1 << 30);
            for (const RowMeta* mm : {&sx, &so, &se}) {
                if (mm->off < 0) continue;
                lo = min(lo, mm->lo);
                hi = max(hi, mm->hi);
            }
            present = lo <= hi;
            lo = max(lo - 1, -n);
            hi = min(hi + 1, m);
        }
        long long off = -1, hoff = -1;
        if (present) {
            const int w = hi - lo + 1;
            off = rs * full_row;
            if (full_hist) {
                hoff = bump;
                bump += ((long long)hbytes * w + (w + 1) / 2 + 15) & ~15LL;
                if (bump > slice_bytes - 16LL * (s + 2)) {
                    if (tid == 0) sh_fail = 1;
                    break;
                }
            }
            RowT* rowM = (RowT*)(slice + off) + n + 1;
            RowT* rowI = rowM + FW;
            RowT* rowD = rowI + FW;
            // Ring cells are addressed from scalar slot bases with 32-bit byte
            // offsets (diagonal k at (k + n + 1) * sizeof(RowT)), so each
            // access is a global load or store with an SGPR base and a VGPR
            // offset, not 64-bit vector address arithmetic.
            unsigned char* wbase = slice + off;
            auto rd = [](const unsigned char* base, uint32_t bo) -> int {
                return *(const RowT*)(base + bo);
            };
            auto wr = [](unsigned char* base, uint32_t bo, RowT v) { *(RowT*)(base + bo) = v; };
            const uint32_t rowb = (uint32_t)FW * (uint32_t)sizeof(RowT);  // bytes per row
            {  // the slot's previous values outside [lo, hi] become NULL
                const int plo = wr_lo[rs], phi = wr_hi[rs];
                for (int k = plo + tid; k <= phi && k < lo; k += BT)
                    rowM[k] = rowI[k] = rowD[k] = (RowT)RNUL;
                for (int k = max(hi + 1, plo) + tid; k <= phi; k += BT)
                    rowM[k] = rowI[k] = rowD[k] = (RowT)RNUL;
            }
            unsigned char* histM = full_hist ? slice + hoff : nullptr;
            uint8_t* histF = full_hist ? histM + (long long)hbytes * w : nullptr;
            // source components (M of s - x and s - o - e, I and D of s - e):
            // the ring slot of step t is t mod R; an absent step reads the
            // NULL slot R
            const int slx = __builtin_amdgcn_readfirstlane(
                sx.off >= 0 ? rs - X + (rs < X ? R : 0) : R);
            const int slo = __builtin_amdgcn_readfirstlane(
                so.off >= 0 ? rs - OE + (rs < OE ? R : 0) : R);
            const int sle = __builtin_amdgcn_readfirstlane(
                se.off >= 0 ? rs - E + (rs < E ? R : 0) : R);
            const unsigned char* MXb = slice + (long long)slx * full_row;
            const unsigned char* MOb = slice + (long long)slo * full_row;
            const unsigned char* IEb = slice + (long long)sle * full_row + rowb;
            const unsigned char* DEb = IEb + rowb;
            // one cell from its five source offsets
            auto cell = [&](int k, int va, int vb, int vc, int ve, int vx) {
                int mval;
                int ival = NUL32, dval = NUL32, rec = 0;
                if (s == 0) {
                    mval = max(k, 0);
                } else {
                    const GenCell c = general_cell(n, m, k, va, vb, vc, ve, vx);
                    mval = c.m;
                    ival = c.i;
                    dval = c.d;
                    if constexpr (HIST) rec = c.rec;
                }
                if (mval >= 0) mval = extend_general(sv, n, m, k, mval);
                const uint32_t bo = (uint32_t)(k + n + 1) * (uint32_t)sizeof(RowT);
                wr(wbase, bo, (RowT)(mval < 0 ? RNUL : mval));
                wr(wbase, bo + rowb, (RowT)(ival < 0 ? RNUL : ival));
                wr(wbase, bo + 2 * rowb, (RowT)(dval < 0 ? RNUL : dval));
                if constexpr (full_hist) {
                    if (h16)
                        ((uint16_t*)histM)[k - lo] = mval < 0 ? (uint16_t)0xFFFF : (uint16_t)mval;
                    else
                        ((int*)histM)[k - lo] = mval;
                    // lanes hold neighbouring diagonals (k - lo has the lane's
                    // parity): both write the byte of the pair of cells; a
                    // partner past hi reads 0
                    const int other = __builtin_amdgcn_update_dpp(0, rec, 0xB1, 0xF, 0xF, false);
                    const int lo4 = (tid & 1) ? other : rec;
                    const int hi4 = (tid & 1) ? rec : other;
                    histF[(k - lo) >> 1] = (uint8_t)(lo4 | (hi4 << 4));
                }
                // an end cell: the last text column with at most pe pattern
                // bases left, or the last pattern row with at most te text
                // bases left (global: the corner cell on diagonal m - n)
                bool at_end;
                if constexpr (FREE)
                    at_end = mval >= 0 && ((mval == m && mval - k >= n - pe) ||
                                           (mval - k == n && mval >= m - te));
                else
                    at_end = k == m - n && mval == m;
                if (at_end) atomicMin(&sh_end, k);
            };
            // two cells per thread and pass: both cells' sources are read
            // before either is computed, so their latencies overlap (a second
            // cell past hi reads in-range sources and is dropped)
            constexpr uint32_t RB = (uint32_t)sizeof(RowT);
            for (int k0 = lo + tid; k0 <= hi; k0 += 2 * BT) {
                const int k1 = k0 + BT;
                const int k1r = min(k1, hi);
                const uint32_t b0 = (uint32_t)(k0 + n + 1) * RB, b1 = (uint32_t)(k1r + n + 1) * RB;
                const int a0 = rd(MOb, b0 - RB), c0 = rd(MOb, b0 + RB), x0 = rd(MXb, b0),
                          i0 = rd(IEb, b0 - RB), e0 = rd(DEb, b0 + RB);
                const int a1 = rd(MOb, b1 - RB), c1 = rd(MOb, b1 + RB), x1 = rd(MXb, b1),
                          i1 = rd(IEb, b1 - RB), e1 = rd(DEb, b1 + RB);
                cell(k0, a0, i0, c0, e0, x0);
                if (k1 <= hi) cell(k1, a1, i1, c1, e1, x1);
            }
        }
        // the range later steps read (the WF-adaptive reduction may narrow it;
        // the step table keeps [lo, hi], by which the history row is indexed)
        int klo = lo, khi = hi;
        if (MWL > 0 && present && hi - lo + 1 >= MWL) {
            __syncthreads();  // every cell written, sh_end final
            if (sh_end == INT_MAX) {  // not for the step that ends the alignment
                RowT* rowM = (RowT*)(slice + off) + n + 1;
                // each thread reads back the cells it wrote (k = lo + tid mod BT)
                int dl = INT_MAX;
                for (int k = lo + tid; k <= hi; k += BT) {
                    const int h = rowM[k];
                    if (h >= 0) dl = min(dl, max(n - (h - k), m - h));
                }
                for (int o2 = 32; o2 >= 1; o2 >>= 1) dl = min(dl, __shfl_xor(dl, o2));
                if ((tid & 63) == 0 && dl != INT_MAX) atomicMin(&sh_dmin, dl);
                __syncthreads();
                const int dmin = sh_dmin;
                if (dmin != INT_MAX) {  // a wavefront without offsets stays as it is
                    int kl = INT_MAX, kh = INT_MIN;
                    for (int k = lo + tid; k <= hi; k += BT) {
                        const int h = rowM[k];
                        if (h >= 0 && max(n - (h - k), m - h) - dmin <= MDT) {
                            kl = min(kl, k);
                            kh = max(kh, k);
                        }
                    }
                    for (int o2 = 32; o2 >= 1; o2 >>= 1) {
                        kl = min(kl, __shfl_xor(kl, o2));
                        kh = max(kh, __shfl_xor(kh, o2));
                    }
                    if ((tid & 63) == 0 && kl != INT_MAX) {
                        atomicMin(&sh_klo, kl);
                        atomicMax(&sh_khi, kh);
                    }
                    __syncthreads();
                    klo = sh_klo;
                    khi = sh_khi;
                    // the dropped diagonals read NULL from now on
                    RowT* rowI = rowM + FW;
                    RowT* rowD = rowI + FW;
                    for (int k = lo + tid; k < klo; k += BT)
                        rowM[k] = rowI[k] = rowD[k] = (RowT)RNUL;
                    for (int k = khi + 1 + tid; k <= hi; k += BT)
                        rowM[k] = rowI[k] = rowD[k] = (RowT)RNUL;
                }
            }
        }
        // this step's metadata (sources of this step are other entries, so
        // no thread still reading them can see it change)
        if (tid == 0) {
            meta[rs] = RowMeta{klo, khi, off};
            // full history: the row's range and place; checkpoint mode: the
            // range later steps read, -1 for no wavefront, -2 for rows not
            // (yet) kept
            if (full_hist) table[-s] = RowMeta{lo, hi, hoff};
            else if (CK) table[-s] = RowMeta{klo, khi, present ? -2LL : -1LL};
        }
        __syncthreads();
        // the slot's range, read by the next step that takes it over (every
        // thread has read this step's entry before the barrier), and the
        // reduction's accumulators, which every thread has read by now
        if (tid == 0 && present) {
            wr_lo[rs] = klo;
            wr_hi[rs] = khi;
        }
        if (tid == 0 && MWL > 0) {
            sh_dmin = INT_MAX;
            sh_klo = INT_MAX;
            sh_khi = INT_MIN;
        }
        if (sh_end != INT_MAX) {
            S = (int)s;
            end_off = off;
            break;
        }
        if (CK && s > 0 && s % CK == 0) {
            // checkpoint: the rows of steps s - R + 1 .. s (all in the ring
            // now), each over the range later steps read, M then I then D
            long long need = 0;
            for (int j = 0; j < R; j++) {
                const long long t = s - R + 1 + j;
                if (t < 0) continue;
                const RowMeta mm = meta[(int)(t % R)];
                if (mm.off >= 0)
                    need += (3LL * (long long)sizeof(RowT) * (mm.hi - mm.lo + 1) + 15) & ~15LL;
            }
            if (bump + need + seg_bytes > slice_bytes - 16LL * (s + 2)) {
                if (tid == 0) sh_fail = 1;
                break;
            }
            for (int j = 0; j < R; j++) {
                const long long t = s - R + 1 + j;
                if (t < 0) continue;
                const RowMeta mm = meta[(int)(t % R)];
                if (mm.off < 0) continue;
                const int w = mm.hi - mm.lo + 1;
                const RowT* src = (const RowT*)(slice + mm.off) + n + 1 + mm.lo;
                RowT* dst = (RowT*)(slice + bump);
                for (int c = 0; c < 3; c++)
                    for (int kk = tid; kk < w; kk += BT) dst[c * w + kk] = src[(long long)c * FW + kk];
                if (tid == 0) table[-t].off = bump;
                bump += (3LL * (long long)sizeof(RowT) * w + 15) & ~15LL;
            }
            __syncthreads();  // copied before the next step takes over the oldest slot
        }
    }
    __syncthreads();
    if (sh_fail == 2) {  // step bound exceeded: give up on the pair, never loop
        if (tid == 0) {
            a.scores[pair] = -1;
            a.nruns[pair] = 0;
            atomicMin(a.gave_up, (unsigned long long)pair);
        }
        return;
    }
    if (sh_fail) {
        if (tid == 0) {
            const uint32_t at = atomicAdd(a.fail_count, 1u);
            a.fail_list[at] = pair;
        }
        return;
    }
    if (!a.cigar) {
        if (tid == 0) {
            a.scores[pair] = S * a.pen.g;
            a.nruns[pair] = 0;
        }
        return;
    }
    // CIGAR mode: the walk runs in its own kernel, one wavefront per pair
    if (tid == 0) a.jstate[job] = GenJobState{bump, end_off, S, sh_end};
}

// The CIGAR backtrace of the general kernel's pairs, one wavefront per pair,
// launched after k_general on the same stream: the forward pass hands over
// the end cell, the score, the end of its history (or checkpoints) and the
// ring offset of the last step.  The walk itself is serial; 64 lanes
// recompute the segments of checkpoint mode.  The forward pass's workgroup
// is free again while the walks run, many per compute unit.
template <bool SEQ_LDS, class RowT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8))) void k_general_walk(
    GeneralArgs a) {
    constexpr int RNUL = sizeof(RowT) == 2 ? -16384 : NUL32;
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ long long sh_ws;
    __shared__ int sh_wk, sh_wstate;

    const uint32_t job = blockIdx.x;
    if (job >= a.num_jobs) return;
    const GenJobState js = a.jstate[job];
    if (js.S < 0) return;  // the forward pass failed or gave up on this pair
    const uint32_t pair = a.jobs[job];
    const PairDesc desc = a.pairs[pair];
    const int n = (int)desc.p_len, m = (int)desc.t_len;
    const int tid = threadIdx.x, BT = blockDim.x;
    const int X = a.pen.x, OE = a.pen.oe, E = a.pen.e, PRE = a.pen.pre;
    const int R = PRE + 1;
    unsigned char* slice = a.arena + a.slice_off[job];
    const long long slice_bytes = (long long)(a.slice_off[job + 1] - a.slice_off[job]);
    const int FW = n + m + 3;
    const long long full_row = (3LL * (long long)sizeof(RowT) * FW + 15) & ~15LL;
    const bool h16 = m < 0xFFFF;
    const int hbytes = h16 ? 2 : 4;
    RowMeta* table = (RowMeta*)(slice + slice_bytes) - 1;
    const int S = js.S, sh_end = js.end_k;
    const long long bump = js.bump, end_off = js.end_off;
    const int CK = a.ckpt;
    const int DMAX = CK ? (CK + R - 1) / E : 0;
    const int WC = 2 * DMAX + 1;
    const long long SEG_ROWB = ((long long)WC * (3 * (long long)sizeof(RowT) + 1) + 15) & ~15LL;
    const long long seg_bytes = CK ? (long long)(CK + R) * SEG_ROWB : 0;

    SeqView<SEQ_LDS> sv;
    const int nwp = (n + 31) >> 5, nwt = (m + 31) >> 5;
    if (CK && SEQ_LDS) {
        uint64_t* p64 = (uint64_t*)lds;
        uint64_t* t64 = p64 + nwp + 1;
        for (int w = tid; w <= nwp; w += BT) p64[w] = w < nwp ? a.pw[desc.p_start + w] : 0ULL;
        for (int w = tid; w <= nwt; w += BT) t64[w] = w < nwt ? a.tw[desc.t_start + w] : 0ULL;
        sv.p = (const uint32_t*)p64;
        sv.t = (const uint32_t*)t64;
        __syncthreads();
    } else {
        sv.p = (const uint32_t*)(a.pw + desc.p_start);
        sv.t = (const uint32_t*)(a.tw + desc.t_start);
    }
    sv.np32 = 2 * nwp;
    sv.nt32 = 2 * nwt;
    (void)hbytes;
    (void)full_row;
    // checkpoint mode: each segment row's diagonal range, in LDS after the
    // staged sequences (the launch sizes the LDS for its longest pair)
    int* seg_a = (int*)(lds + (CK && SEQ_LDS ? (((nwp + 1 + nwt + 1) * 8 + 15) & ~15) : 0));
    int* seg_b = seg_a + (CK + R);

    if (CK) {
        // ---- checkpoint mode: the backtrace, one segment at a time --------
        // The walk starts at the end cell and runs back over a segment of
        // steps (b, se], recomputed first from the checkpoint at step b (b a
        // multiple of CK; b = 0: from the start) in the cone of diagonals
        // that can reach the entry cell (se, ke): a step t's cells lie within
        // (se - t) / e diagonals of ke, since every change of diagonal costs at
        // least e.  The cone holds every source of its own cells, so each
        // recomputed cell equals the forward pass's.  When the walk reaches a
        // step at or below b, that cell is the entry of the next segment.
        unsigned char* segbuf = slice + bump;
        const long long runs_at = bump + seg_bytes;
        uint32_t* out = (uint32_t*)(slice + runs_at);
        const long long table_bottom = slice_bytes - 16LL * (S + 1);
        const long long cap_runs = (table_bottom - runs_at) / 4;
        long long nr = 0;
        int cop = -1;
        long long clen = 0;
        auto emit = [&](int op, long long len) {
            if (len <= 0) return;
            if (op == cop) {
                clen += len;
            } else {
                if (cop >= 0) {
                    if (nr < cap_runs) out[nr] = ((uint32_t)clen << 4) | (uint32_t)cop;
                    nr++;
                }
                cop = op;
                clen = len;
            }
        };
        // the walk's state (thread 0): step, diagonal, offset, component
        // (0 M, 1 I, 2 D)
        long long ws = S;
        int wk = sh_end, wh = 0, wc = 0;
        if (tid == 0) {
            wh = ((const RowT*)(slice + end_off) + n + 1)[wk];
            emit(OP_D, n - (wh - wk));  // the free suffix (runs go last to first)
            emit(OP_I, m - wh);
            sh_ws = S;
            sh_wk = sh_end;
            sh_wstate = 0;
        }
        __syncthreads();
        for (;;) {
            const long long se = sh_ws;
            const int ke = sh_wk, state = sh_wstate;
            __syncthreads();  // read before thread 0 writes the next hand-over
            if (state != 0) break;
            const long long b = se > 0 ? ((se - 1) / CK) * CK : 0;
            const long long t0 = b > 0 ? b - R + 1 : 0;
            const int nrow = (int)(se - t0 + 1);
            const int kb = ke - DMAX;  // diagonal of column 0
            for (int r = tid; r < nrow; r += BT) {
                const long long t = t0 + r;
                const RowMeta mm = table[-t];
                const int dl = (int)((se - t) / E);
                seg_a[r] = mm.off == -1 ? 1 : max(ke - dl, mm.lo);
                seg_b[r] = mm.off == -1 ? 0 : min(ke + dl, mm.hi);
            }
            __syncthreads();
            // the segment buffer: per row M, I, D (WC columns each) and the
            // decision records
            auto rowp = [&](int r) -> RowT* { return (RowT*)(segbuf + (long long)r * SEG_ROWB); };
            auto src = [&](long long ts, int comp, int kk) -> int {
                if (ts < t0) return RNUL;
                const int rr = (int)(ts - t0);
                if (kk < seg_a[rr] || kk > seg_b[rr]) return RNUL;
                return rowp(rr)[comp * WC + (kk - kb)];
            };
            // Every row holds NULL on the cone's columns outside its cells, so
            // the recomputed cells read their sources without range tests: a
            // source of step t' lies in the cone of t' (one more diagonal per
            // e steps back), within the row's WC columns.
            auto pad_row = [&](int r) {
                const int dl = (int)((se - (t0 + r)) / E);
                const int ca = ke - dl, cb = ke + dl;
                const int sa = seg_a[r], sb = seg_b[r];
                RowT* row = rowp(r);
                const int na = sa <= sb ? min(sa, cb + 1) : cb + 1;  // [ca, na) before the cells
                for (int kk = ca + tid; kk < na; kk += BT)
                    row[kk - kb] = row[WC + kk - kb] = row[2 * WC + kk - kb] = (RowT)RNUL;
                for (int kk = (sa <= sb ? max(sb + 1, ca) : cb + 1) + tid; kk <= cb; kk += BT)
                    row[kk - kb] = row[WC + kk - kb] = row[2 * WC + kk - kb] = (RowT)RNUL;
            };
            auto src_in_cone = [&](long long ts, int comp, int kk) -> int {
                if (ts < t0) return RNUL;
                return rowp((int)(ts - t0))[comp * WC + (kk - kb)];
            };
            if (b > 0) {  // the checkpoint's rows, within the cone
                for (int r = 0; r < R; r++) {
                    pad_row(r);
                    const int lo_ = seg_a[r], hi_ = seg_b[r];
                    if (lo_ > hi_) continue;
                    const RowMeta mm = table[-(t0 + r)];
                    const int w = mm.hi - mm.lo + 1, cnt = hi_ - lo_ + 1;
                    const RowT* from = (const RowT*)(slice + mm.off);
                    RowT* to = rowp(r);
                    for (int c = 0; c < 3; c++)
                        for (int kk = lo_ + tid; kk <= hi_; kk += BT)
                            to[c * WC + (kk - kb)] = from[(long long)c * w + (kk - mm.lo)];
                }
                __syncthreads();  // the first recomputed step reads these rows
            }
            for (long long t = b > 0 ? b + 1 : 0; t <= se; t++) {
                const int r = (int)(t - t0);
                RowT* dM = rowp(r);
                uint8_t* dF = (uint8_t*)(dM + 3 * WC);
                pad_row(r);
                for (int k = seg_a[r] + tid; k <= seg_b[r]; k += BT) {
                    int mval, ival = NUL32, dval = NUL32, rec = 0;
                    if (t == 0) {
                        mval = max(k, 0);
                    } else {
                        const GenCell c = general_cell(
                            n, m, k, src_in_cone(t - OE, 0, k - 1), src_in_cone(t - E, 1, k - 1),
                            src_in_cone(t - OE, 0, k + 1), src_in_cone(t - E, 2, k + 1),
                            src_in_cone(t - X, 0, k));
                        mval = c.m;
                        ival = c.i;
                        dval = c.d;
                        rec = c.rec;
                    }
                    if (mval >= 0) mval = extend_general(sv, n, m, k, mval);
                    dM[k - kb] = (RowT)(mval < 0 ? RNUL : mval);
                    dM[WC + k - kb] = (RowT)(ival < 0 ? RNUL : ival);
                    dM[2 * WC + k - kb] = (RowT)(dval < 0 ? RNUL : dval);
                    dF[k - kb] = (uint8_t)rec;
                }
                __syncthreads();
            }
            if (tid == 0) {
                auto val = [&](long long ts, int comp, int kk) -> int {
                    const int v = src(ts, comp, kk);
                    return v < 0 ? NUL32 : v;
                };
                int st = 0;  // 0: next segment, 1: done, 2: inconsistent
                for (;;) {
                    if (ws < 0 || wh < 0) {
                        st = 2;
                        break;
                    }
                    if (ws == 0) {  // M_0[k] = max(k, 0) before extension, after the free prefix
                        if (wc != 0) {
                            st = 2;
                            break;
                        }
                        emit(OP_M, wh - max(wk, 0));
                        emit(OP_I, wk);
                        emit(OP_D, -wk);
                        st = 1;
                        break;
                    }
                    if (ws <= b) break;  // below this segment: hand over
                    const int rr = (int)(ws - t0);
                    if (wk < seg_a[rr] || wk > seg_b[rr]) {
                        st = 2;
                        break;
                    }
                    const int f = ((const uint8_t*)(rowp(rr) + 3 * WC))[wk - kb];
                    if (wc == 0) {
                        const int ms = f & 3;
                        if (ms == 0) {
                            const int hn = val(ws - X, 0, wk);
                            if (hn < 0 || hn + 1 > wh) {
                                st = 2;
                                break;
                            }
                            emit(OP_M, wh - hn - 1);
                            emit(OP_X, 1);
                            ws -= X;
                            wh = hn;
                        } else {
                            const int h0 = val(ws, ms, wk);  // I or D before the M cell
                            if (h0 < 0 || h0 > wh) {
                                st = 2;
                                break;
                            }
                            emit(OP_M, wh - h0);
                            wh = h0;
                            wc = ms;
                        }
                    } else if (wc == 1) {  // insertion: from k - 1, one text base
                        emit(OP_I, 1);
                        wk -= 1;
                        wh -= 1;
                        if (f & 4) {
                            ws -= OE;
                            wc = 0;
                        } else {
                            ws -= E;
                        }
                    } else {  // deletion: from k + 1, one pattern base
                        emit(OP_D, 1);
                        wk += 1;
                        if (f & 8) {
                            ws -= OE;
                            wc = 0;
                        } else {
                            ws -= E;
                        }
                    }
                }
                sh_ws = ws;
                sh_wk = wk;
                sh_wstate = st;
            }
            __syncthreads();
        }
        if (tid != 0) return;
        if (sh_wstate == 2) {  // inconsistent walk: give up on the pair, no loop
            a.scores[pair] = -1;
            a.nruns[pair] = 0;
            atomicMin(a.gave_up, (unsigned long long)pair);
            return;
        }
        if (cop >= 0) {
            if (nr < cap_runs) out[nr] = ((uint32_t)clen << 4) | (uint32_t)cop;
            nr++;
        }
        if (nr > cap_runs) {
            const uint32_t at = atomicAdd(a.fail_count, 1u);
            a.fail_list[at] = pair;
            return;
        }
        a.scores[pair] = S * a.pen.g;
        a.nruns[pair] = (uint32_t)nr;
        a.job_nruns[job] = (uint32_t)nr;
        a.job_used[job] =
            (uint64_t)(bump - (R + 1) * full_row + seg_bytes) + 16ull * (S + 1) + 4ull * nr;
        a.run_src[pair] = (a.slice_off[job] + (uint64_t)runs_at) / 4;  // arena words
        return;
    }
    // backtrace by one thread over the step table and the history rows, one
    // event per iteration (as in the short kernel)
    if (tid != 0) return;
    uint32_t* out = (uint32_t*)(slice + bump);
    const long long table_bottom = slice_bytes - 16LL * (S + 1);
    const long long cap_runs = (table_bottom - bump) / 4;
    long long nr = 0;
    int cop = -1;
    long long clen = 0;
    auto emit = [&](int op, long long len) {
        if (len <= 0) return;
        if (op == cop) {
            clen += len;
        } else {
            if (cop >= 0) {
                if (nr < cap_runs) out[nr] = ((uint32_t)clen << 4) | (uint32_t)cop;
                nr++;
            }
            cop = op;
            clen = len;
        }
    };
    // M offset after extension of (ss, kk), NULL outside the step's range
    auto getM = [&](long long ss, int kk) -> int {
        if (ss < 0) return NUL32;
        const RowMeta mm = table[-ss];
        if (mm.off < 0 || kk < mm.lo || kk > mm.hi) return NUL32;
        if (h16) {
            const uint16_t v = ((const uint16_t*)(slice + mm.off))[kk - mm.lo];
            return v == 0xFFFF ? NUL32 : (int)v;
        }
        return ((const int*)(slice + mm.off))[kk - mm.lo];
    };
    // decision record of (ss, kk); -1 outside the step's range
    auto getF = [&](long long ss, int kk) -> int {
        if (ss <= 0) return -1;
        const RowMeta mm = table[-ss];
        if (mm.off < 0 || kk < mm.lo || kk > mm.hi) return -1;
        const int w = mm.hi - mm.lo + 1;
        const uint8_t* f = (const uint8_t*)(slice + mm.off) + (long long)hbytes * w;
        return (f[(kk - mm.lo) >> 1] >> (((kk - mm.lo) & 1) << 2)) & 15;
    };
    long long s = S;
    int k = sh_end, h = getM(S, k);
    // the free suffix (runs are emitted last to first)
    emit(OP_D, n - (h - k));
    emit(OP_I, m - h);
    bool bad = false;
    for (;;) {
        if (s < 0 || h < 0) {
            bad = true;
            break;
        }
        if (s == 0) {  // M_0[k] = max(k, 0) before extension, after the free prefix
            emit(OP_M, h - max(k, 0));
            emit(OP_I, k);
            emit(OP_D, -k);
            break;
        }
        const int f = getF(s, k);
        if (f < 0) {
            bad = true;
            break;
        }
        const int ms = f & 3;
        int hn, h0, L = 1, dk = 0;
        long long s2;
        if (ms == 0) {
            hn = getM(s - X, k);
            h0 = hn + 1;
            s2 = s - X;
        } else {
            // follow the gap back along its chain to where it opened from M
            const int bit = ms == 1 ? 4 : 8;
            const int dj = ms == 1 ? -1 : 1;
            long long sc = s;
            int kc = k, fc = f;
            while (fc >= 0 && !(fc & bit)) {
                sc -= E;
                kc += dj;
                L++;
                fc = getF(sc, kc);
            }
            if (fc < 0) {
                bad = true;
                break;
            }
            hn = getM(sc - OE, kc + dj);
            h0 = ms == 1 ? hn + L : hn;  // insertions consume text
            s2 = sc - OE;
            dk = dj * L;
        }
        if (hn < 0 || h0 > h) {
            bad = true;
            break;
        }
        emit(OP_M, h - h0);
        emit(ms + 1, L);  // op codes: X=1 I=2 D=3
        s = s2;
        k += dk;
        h = hn;
    }
    if (bad) {  // inconsistent walk: give up on the pair, no loop
        a.scores[pair] = -1;
        a.nruns[pair] = 0;
        atomicMin(a.gave_up, (unsigned long long)pair);
        return;
    }
    if (cop >= 0) {
        if (nr < cap_runs) out[nr] = ((uint32_t)clen << 4) | (uint32_t)cop;
        nr++;
    }
    if (nr > cap_runs) {
        const uint32_t at = atomicAdd(a.fail_count, 1u);
        a.fail_list[at] = pair;
        return;
    }
    a.scores[pair] = S * a.pen.g;
    a.nruns[pair] = (uint32_t)nr;
    a.job_nruns[job] = (uint32_t)nr;
    a.job_used[job] = (uint64_t)(bump - (R + 1) * full_row) + 16ull * (S + 1) + 4ull * nr;
    a.run_src[pair] = (a.slice_off[job] + (uint64_t)bump) / 4;  // arena words
}

// Move the runs of finished general jobs out of the arena.
__global__ void k_gather_general(const uint32_t* __restrict__ jobs, size_t njobs,
                                 const uint32_t* __restrict__ nruns, uint64_t* __restrict__ run_src,
                                 const uint32_t* __restrict__ arena32,
                                 const uint64_t* __restrict__ job_offsets, uint64_t gen_base,
                                 uint32_t* __restrict__ gen_runs) {
    const size_t j = blockIdx.x;
    if (j >= njobs) return;
    const uint32_t pair = jobs[j];
    const uint64_t src = run_src[pair];
    const uint64_t dst = gen_base + job_offsets[j];
    const uint32_t cnt = nruns[j];  // per job; 0 for jobs that failed
    if (cnt == 0) return;
    for (uint32_t r = threadIdx.x; r < cnt; r += blockDim.x) gen_runs[dst + r] = arena32[src + r];
    __syncthreads();
    if (threadIdx.x == 0) run_src[pair] = GEN_BIT | dst;
}

__global__ void k_pair_lengths(const PairDesc* __restrict__ pairs, const uint32_t* __restrict__ idx,
                               size_t n, uint32_t* __restrict__ out) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const PairDesc d = pairs[idx[i]];
        out[2 * i] = d.p_len;
        out[2 * i + 1] = d.t_len;
    }
}

// reversed runs -> caller buffer in alignment order (nothing is written if
// the total exceeds the capacity).  A block takes COMPACT_PAIRS consecutive
// pairs and fills their whole output range [offsets[first], offsets[first +
// COMPACT_PAIRS]) with consecutive threads on consecutive runs, so every
// store is coalesced.  The pair of each output position comes from an LDS
// table that every pair's thread fills over its own range (one byte per run,
// the pair's index in the tile); a tile with more runs than the table holds
// finds it by a binary search over the run ends instead.  A pair's runs sit
// in its slot in backtrace order, so position q takes slot entry end - 1 - q.
// Reads stay scattered across pairs (slots follow the bucketed order), but a
// wave's 64 positions touch only the few pairs they belong to.
constexpr int COMPACT_PAIRS = 256;
constexpr int COMPACT_UNROLL = 4;
constexpr int COMPACT_OWNER = 16384;

__global__ __launch_bounds__(COMPACT_PAIRS) void k_compact(const uint64_t* __restrict__ run_src,
                                                           const uint32_t* __restrict__ slots,
                                                           const uint32_t* __restrict__ slots2,
                                                           const uint32_t* __restrict__ gen_runs,
                                                           const uint64_t* __restrict__ offsets,
                                                           size_t n, uint32_t* __restrict__ out,
                                                           uint64_t capacity,
                                                           uint64_t* __restrict__ total_out) {
    __shared__ uint64_t end[COMPACT_PAIRS];
    __shared__ const uint32_t* src_of[COMPACT_PAIRS];
    __shared__ uint8_t owner[COMPACT_OWNER];
    if (total_out && blockIdx.x == 0 && threadIdx.x == 0) *total_out = offsets[n];
    if (offsets[n] > capacity) return;
    const int t = threadIdx.x;
    const size_t tiles = (n + COMPACT_PAIRS - 1) / COMPACT_PAIRS;
    for (size_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const size_t first = tile * COMPACT_PAIRS;
        const int np = (int)min((size_t)COMPACT_PAIRS, n - first);
        const uint64_t lo = offsets[first], hi = offsets[first + np];
        const bool table = hi - lo <= (uint64_t)COMPACT_OWNER;
        if (t < np) {
            const uint64_t src = run_src[first + t];
            const uint64_t off = src & ~(GEN_BIT | SLOTS2_BIT);
            src_of[t] = (src & GEN_BIT) ? gen_runs + off : ((src & SLOTS2_BIT) ? slots2 : slots) + off;
            const uint64_t e = offsets[first + t + 1];
            end[t] = e;
            if (table)
                for (uint32_t r = (uint32_t)(offsets[first + t] - lo); r < (uint32_t)(e - lo); r++)
                    owner[r] = (uint8_t)t;
        }
        __syncthreads();
        if (table) {
            const uint32_t total = (uint32_t)(hi - lo);
            for (uint32_t q0 = t; q0 < total; q0 += COMPACT_PAIRS * COMPACT_UNROLL) {
                uint32_t v[COMPACT_UNROLL];
#pragma unroll
                for (int u = 0; u < COMPACT_UNROLL; u++) {
                    const uint32_t q = q0 + (uint32_t)u * COMPACT_PAIRS;
                    if (q < total) {
                        const int p = owner[q];
                        v[u] = src_of[p][(uint32_t)(end[p] - lo) - 1 - q];
                    }
                }
#pragma unroll
                for (int u = 0; u < COMPACT_UNROLL; u++) {
                    const uint32_t q = q0 + (uint32_t)u * COMPACT_PAIRS;
                    if (q < total) out[lo + q] = v[u];
                }
            }
        } else {
            for (uint64_t q0 = lo + t; q0 < hi; q0 += COMPACT_PAIRS * COMPACT_UNROLL) {
                uint32_t v[COMPACT_UNROLL];
#pragma unroll
                for (int u = 0; u < COMPACT_UNROLL; u++) {
                    const uint64_t q = q0 + (uint64_t)u * COMPACT_PAIRS;
                    if (q < hi) {
                        // p = number of tile pairs whose runs end at or before q
                        // (ends never decrease); q < hi keeps p below np
                        int p = 0;
#pragma unroll
                        for (int step = COMPACT_PAIRS / 2; step; step >>= 1)
                            if (p + step <= np && end[p + step - 1] <= q) p += step;
                        v[u] = src_of[p][end[p] - 1 - q];
                    }
                }
#pragma unroll
                for (int u = 0; u < COMPACT_UNROLL; u++) {
                    const uint64_t q = q0 + (uint64_t)u * COMPACT_PAIRS;
                    if (q < hi) out[q] = v[u];
                }
            }
        }
        __syncthreads();
    }
}

// Bucket key: longer pairs and larger length differences (more expected
// work) first, so a persistent grid starts the long jobs early and lane
// groups sharing a wave hold pairs of similar cost.
__device__ __forceinline__ uint32_t bucket_key(const PairDesc& d) {
    const uint32_t p = d.p_len, t = d.t_len;
    const uint32_t len = max(p, t), diff = p > t ? p - t : t - p;
    const uint32_t k = min(len >> 5, 63u) * 64u + min(diff, 63u);
    return (BUCKET_KEYS - 1) - k;
}

// Each block owns BUCKET_CHUNK consecutive pairs.  Counting goes through an
// LDS histogram first, so the global histogram sees one atomic per
// (block, key) instead of one per pair.
constexpr int BUCKET_CHUNK = 8192;

__global__ __launch_bounds__(256) void k_bucket_keys(const PairDesc* __restrict__ pairs, size_t n,
                                                     uint32_t* __restrict__ keys,
                                                     uint32_t* __restrict__ hist) {
    __shared__ uint32_t local[BUCKET_KEYS];
    for (int i = threadIdx.x; i < BUCKET_KEYS; i += blockDim.x) local[i] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * BUCKET_CHUNK;
    const size_t end = min(n, base + BUCKET_CHUNK);
    for (size_t i = base + threadIdx.x; i < end; i += blockDim.x) {
        const uint32_t key = bucket_key(pairs[i]);
        keys[i] = key;
        atomicAdd(&local[key], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < BUCKET_KEYS; i += blockDim.x)
        if (local[i]) atomicAdd(&hist[i], local[i]);
}

// Each block takes the exclusive scan of the whole histogram (the first
// pair of each key's range) into LDS, reserves one range per key it holds
// by adding its count to `taken` (the pairs of that key placed so far), and
// places its pairs inside those ranges.
constexpr int BUCKET_PER_THREAD = BUCKET_KEYS / 256;
__global__ __launch_bounds__(256) void k_bucket_scatter(const uint32_t* __restrict__ keys, size_t n,
                                                        const uint32_t* __restrict__ hist,
                                                        uint32_t* __restrict__ taken,
                                                        uint32_t* __restrict__ order) {
    __shared__ uint32_t count[BUCKET_KEYS];
    __shared__ uint32_t start[BUCKET_KEYS];
    const int t = threadIdx.x;
    for (int i = t; i < BUCKET_KEYS; i += 256) count[i] = 0;
    {
        uint32_t h[BUCKET_PER_THREAD];
        uint64_t own = 0;
#pragma unroll
        for (int j = 0; j < BUCKET_PER_THREAD; j++) {
            h[j] = hist[t * BUCKET_PER_THREAD + j];
            own += h[j];
        }
        uint64_t incl = own;
        block_inclusive_scan(incl);
        uint32_t run = (uint32_t)(incl - own);
#pragma unroll
        for (int j = 0; j < BUCKET_PER_THREAD; j++) {
            start[t * BUCKET_PER_THREAD + j] = run;
            run += h[j];
        }
    }
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * BUCKET_CHUNK;
    const size_t end = min(n, base + BUCKET_CHUNK);
    for (size_t i = base + t; i < end; i += 256) atomicAdd(&count[keys[i]], 1u);
    __syncthreads();
    for (int i = t; i < BUCKET_KEYS; i += 256) {
        if (count[i]) start[i] += atomicAdd(&taken[i], count[i]);
        count[i] = 0;
    }
    __syncthreads();
    for (size_t i = base + t; i < end; i += 256) {
        const uint32_t key = keys[i];
        const uint32_t r = atomicAdd(&count[key], 1u);
        order[start[key] + r] = (uint32_t)i;
    }
}

__global__ void k_scores_fail(const uint32_t* list, size_t n, int32_t* scores) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        scores[list[i]] = -1;
}

int grid_for(size_t n, int block, int max_blocks = 65536) {
    size_t b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > (size_t)max_blocks) b = max_blocks;
    return (int)b;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_batch_stats(const PairDesc* pairs, size_t n, BatchStats* out, uint32_t max_len,
                              hipStream_t s) {
    // out[1 .. STATS_BLOCKS] hold the per-block partials
    const int nb = n ? grid_for(n, 256 * 8, STATS_BLOCKS) : 1;
    hipLaunchKernelGGL(k_batch_stats, dim3(nb), dim3(256), 0, s, pairs, n, out + 1, max_len);
    hipLaunchKernelGGL(k_batch_stats_final, dim3(1), dim3(256), 0, s, out + 1, nb, out);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_multi(const FillOps& ops, hipStream_t s) {
    if (ops.count < 0 || ops.count > FILL_OPS) return hipErrorInvalidValue;
    uint64_t total = 0;
    for (int o = 0; o < ops.count; o++) total += ops.op[o].n;
    if (total)
        hipLaunchKernelGGL(k_fill_multi, dim3(grid_for((total + 3) / 4, 256, 2048)), dim3(256), 0, s,
                           ops);
    return hipGetLastError();
}

hipError_t launch_add_u64(const uint64_t* src, uint64_t add, size_t n, uint64_t* dst,
                          hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_add_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, src, add, n, dst);
    return hipGetLastError();
}

size_t scan_temp_bytes(size_t n) { return ((n + SCAN_TILE - 1) / SCAN_TILE + 1) * sizeof(uint64_t); }

hipError_t launch_scan(ScanKind kind, const void* in, size_t n, uint64_t* out, void* temp,
                       hipStream_t s) {
    const size_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    uint64_t* bs = (uint64_t*)temp;
    if (nb == 0) {
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, out, 0ull, (size_t)1);
        return hipGetLastError();
    }
    if (n <= SCAN_SINGLE_MAX) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(SCAN_T), 0, s, kind, in, n, out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_partial, dim3(nb), dim3(SCAN_T), 0, s, kind, in, n, bs);
    const int prefixed = nb > SCAN_SELF_MAX ? 1 : 0;
    if (prefixed) hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(SCAN_T), 0, s, bs, nb);
    hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(SCAN_T), 0, s, kind, in, n, bs, prefixed, out);
    return hipGetLastError();
}

hipError_t launch_pack_pairs(const PairDesc* pairs, size_t n, const uint8_t* pascii,
                             const uint8_t* tascii, const uint64_t* ws_p, const uint64_t* ws_t,
                             uint32_t max_words_p, uint32_t max_words_t, uint64_t* words_p,
                             uint64_t* words_t, PairDesc* packed_pairs, unsigned long long* err_pair,
                             hipStream_t s) {
    const uint32_t mw = max(max(max_words_p, max_words_t), 1u);
    const size_t total = n * (size_t)mw;
    if (n)
        hipLaunchKernelGGL(k_pack_pairs, dim3(grid_for(total, 256, 1 << 19), 2), dim3(256), 0, s,
                           pairs, n, pascii, tascii, ws_p, ws_t, max(max_words_p, 1u),
                           max(max_words_t, 1u), words_p, words_t, packed_pairs, err_pair);
    return hipGetLastError();
}

hipError_t launch_pack_seqs(const uint8_t* ascii, const uint64_t* starts, const uint32_t* lens,
                            size_t n, const uint64_t* word_starts, uint64_t total_words,
                            uint64_t* words, unsigned long long* err_index, hipStream_t s) {
    if (n && total_words)
        hipLaunchKernelGGL(k_pack_seqs, dim3(grid_for(total_words, 256, 1 << 20)), dim3(256), 0, s,
                           ascii, starts, lens, n, word_starts, total_words, words, err_index);
    return hipGetLastError();
}

int short_groups_per_block(int lanes, int block_threads) {
    return (block_threads / 64) * (64 / lanes);
}

template <int G, int DPL, class RowT>
static hipError_t launch_short_t(const ShortArgs& a, bool cigar, bool persistent, int bt, int grid,
                                 hipStream_t s) {
    const size_t lds = (size_t)short_groups_per_block(G, bt) * a.group_bytes;
    const bool ends = a.ends.pb || a.ends.pe || a.ends.tb || a.ends.te;
    const int pers = persistent ? 1 : 0;
    if (cigar && ends)
        hipLaunchKernelGGL((k_short<G, DPL, true, RowT, true>), dim3(grid), dim3(bt), lds, s, a, pers);
    else if (cigar)
        hipLaunchKernelGGL((k_short<G, DPL, true, RowT, false>), dim3(grid), dim3(bt), lds, s, a, pers);
    else if (ends)
        hipLaunchKernelGGL((k_short<G, DPL, false, RowT, true>), dim3(grid), dim3(bt), lds, s, a, pers);
    else
        hipLaunchKernelGGL((k_short<G, DPL, false, RowT, false>), dim3(grid), dim3(bt), lds, s, a, pers);
    return hipGetLastError();
}

template <int G, int DPL, class RowT>
static int occ_t(bool cigar, int bt, int lds) {
    // the ends-free variants hold the same LDS and launch bounds
    int blocks = 0;
    hipError_t e = cigar ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                               &blocks, (const void*)k_short<G, DPL, true, RowT, false>, bt, lds)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                               &blocks, (const void*)k_short<G, DPL, false, RowT, false>, bt, lds);
    return e == hipSuccess ? blocks : 0;
}

// (window, lanes per pair) shapes the short kernel is built for
#define WFA_SHORT_SHAPES(X) \
    X(16, 8, 2)             \
    X(16, 16, 1)            \
    X(24, 8, 3)             \
    X(32, 8, 4)             \
    X(32, 32, 1)            \
    X(32, 16, 2)            \
    X(48, 16, 3)            \
    X(64, 64, 1)            \
    X(64, 32, 2)            \
    X(64, 16, 4)            \
    X(128, 64, 2)           \
    X(128, 32, 4)           \
    X(256, 64, 4)

bool short_shape_supported(int window, int lanes) {
#define WFA_CASE(w, g, dpl) \
    if (window == w && lanes == g) return true;
    WFA_SHORT_SHAPES(WFA_CASE)
#undef WFA_CASE
    return false;
}

template <class RowT>
static hipError_t launch_short_w(const ShortArgs& a, int window, int lanes, bool cigar,
                                 bool persistent, int bt, int grid, hipStream_t s) {
#define WFA_CASE(w, g, dpl) \
    if (window == w && lanes == g) return launch_short_t<g, dpl, RowT>(a, cigar, persistent, bt, grid, s);
    WFA_SHORT_SHAPES(WFA_CASE)
#undef WFA_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_short(const ShortArgs& a, int window, int lanes, bool cigar, bool persistent,
                        int block_threads, int grid, hipStream_t s) {
    if (a.row_bytes == 1)
        return launch_short_w<int8_t>(a, window, lanes, cigar, persistent, block_threads, grid, s);
    return launch_short_w<int16_t>(a, window, lanes, cigar, persistent, block_threads, grid, s);
}

template <class RowT>
static int occ_w(int window, int lanes, bool cigar, int bt, int lds) {
#define WFA_CASE(w, g, dpl) \
    if (window == w && lanes == g) return occ_t<g, dpl, RowT>(cigar, bt, lds);
    WFA_SHORT_SHAPES(WFA_CASE)
#undef WFA_CASE
    return 0;
}

int short_max_blocks_per_cu(int window, int lanes, bool cigar, int bt, int lds_per_block,
                            int row_bytes) {
    return row_bytes == 1 ? occ_w<int8_t>(window, lanes, cigar, bt, lds_per_block)
                          : occ_w<int16_t>(window, lanes, cigar, bt, lds_per_block);
}

hipError_t launch_general(const GeneralArgs& a, int block_threads, bool seq_in_lds, int lds_bytes,
                          bool rows16, hipStream_t s) {
    if (!a.num_jobs) return hipSuccess;
    const dim3 grid(a.num_jobs), walk(64);
    const int ml = general_meta_lds(a.pen.pre + 1);
    const int fl = seq_in_lds ? ml + lds_bytes : ml;
    const bool hist = a.cigar && a.ckpt == 0;
    const bool free_ends = (a.ends.pb | a.ends.pe | a.ends.tb | a.ends.te) != 0;
#define WFA_GEN_LAUNCH(SL, RT, H, F) \
    hipLaunchKernelGGL((k_general<SL, RT, H, F>), grid, dim3(block_threads), fl, s, a)
#define WFA_GEN_LAUNCH2(SL, RT, H) \
    if (free_ends) WFA_GEN_LAUNCH(SL, RT, H, true); else WFA_GEN_LAUNCH(SL, RT, H, false)
    if (seq_in_lds && rows16) {
        if (hist) { WFA_GEN_LAUNCH2(true, int16_t, true); } else { WFA_GEN_LAUNCH2(true, int16_t, false); }
    } else if (seq_in_lds) {
        if (hist) { WFA_GEN_LAUNCH2(true, int32_t, true); } else { WFA_GEN_LAUNCH2(true, int32_t, false); }
    } else if (rows16) {
        if (hist) { WFA_GEN_LAUNCH2(false, int16_t, true); } else { WFA_GEN_LAUNCH2(false, int16_t, false); }
    } else {
        if (hist) { WFA_GEN_LAUNCH2(false, int32_t, true); } else { WFA_GEN_LAUNCH2(false, int32_t, false); }
    }
#undef WFA_GEN_LAUNCH2
#undef WFA_GEN_LAUNCH
    if (!a.cigar) return hipGetLastError();
    // the walks, one wavefront per pair; checkpoint mode stages the sequences
    // in LDS as the forward pass did, followed by its segment rows' ranges
    const bool walk_lds = seq_in_lds && a.ckpt > 0;
    const int segs = a.ckpt > 0 ? 8 * (a.ckpt + a.pen.pre + 1) : 0;
    const int wl = (walk_lds ? ((lds_bytes + 15) & ~15) : 0) + segs;
    if (walk_lds && rows16)
        hipLaunchKernelGGL((k_general_walk<true, int16_t>), grid, walk, wl, s, a);
    else if (walk_lds)
        hipLaunchKernelGGL((k_general_walk<true, int32_t>), grid, walk, wl, s, a);
    else if (rows16)
        hipLaunchKernelGGL((k_general_walk<false, int16_t>), grid, walk, wl, s, a);
    else
        hipLaunchKernelGGL((k_general_walk<false, int32_t>), grid, walk, wl, s, a);
    return hipGetLastError();
}

hipError_t launch_gather_general(const uint32_t* jobs, size_t njobs, const uint32_t* nruns,
                                 uint64_t* run_src, const uint8_t* arena, uint64_t slice_bytes,
                                 const uint64_t* job_offsets, uint64_t gen_base,
                                 uint32_t* gen_runs, hipStream_t s) {
    (void)slice_bytes;
    if (njobs)
        hipLaunchKernelGGL(k_gather_general, dim3(njobs), dim3(256), 0, s, jobs, njobs, nruns,
                           run_src, (const uint32_t*)arena, job_offsets, gen_base, gen_runs);
    return hipGetLastError();
}

hipError_t launch_pair_lengths(const PairDesc* pairs, const uint32_t* idx, size_t n, uint32_t* out,
                               hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_pair_lengths, dim3(grid_for(n, 256)), dim3(256), 0, s, pairs, idx, n, out);
    return hipGetLastError();
}

hipError_t launch_compact(const uint64_t* run_src, const uint32_t* slots, const uint32_t* slots2,
                          const uint32_t* gen_runs, const uint64_t* offsets, size_t n,
                          uint32_t* out, uint64_t capacity, uint64_t* total_out, hipStream_t s) {
    if (n)
        hipLaunchKernelGGL(k_compact, dim3(grid_for(n, COMPACT_PAIRS, 1 << 20)), dim3(COMPACT_PAIRS),
                           0, s, run_src, slots, slots2, gen_runs, offsets, n, out, capacity,
                           total_out);
    return hipGetLastError();
}

hipError_t launch_bucket_keys(const PairDesc* pairs, size_t n, uint32_t* keys, uint32_t* hist,
                              hipStream_t s) {
    const size_t blocks = (n + BUCKET_CHUNK - 1) / BUCKET_CHUNK;
    if (n)
        hipLaunchKernelGGL(k_bucket_keys, dim3(blocks), dim3(256), 0, s, pairs, n, keys, hist);
    return hipGetLastError();
}

hipError_t launch_bucket_scatter(const uint32_t* keys, size_t n, const uint32_t* hist,
                                 uint32_t* taken, uint32_t* order, hipStream_t s) {
    const size_t blocks = (n + BUCKET_CHUNK - 1) / BUCKET_CHUNK;
    if (n)
        hipLaunchKernelGGL(k_bucket_scatter, dim3(blocks), dim3(256), 0, s, keys, n, hist, taken,
                           order);
    return hipGetLastError();
}

hipError_t launch_scatter_scores_fail(const uint32_t* list, size_t n, int32_t* scores,
                                      hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_scores_fail, dim3(grid_for(n, 256)), dim3(256), 0, s, list, n, scores);
    return hipGetLastError();
}

}  // namespace wfa
