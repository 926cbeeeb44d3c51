// One lane per pair: the wavefront algorithm with every wavefront row of a
// pair in registers, for short reads under a fixed penalty set.
//
// The paper runs one pair per DPU thread (Introduction and Methods); on a
// GPU the same independence puts one pair on each lane of a wavefront, 64
// pairs stepping through the score steps together.  What makes this pay on
// CDNA is that, for fixed scaled penalties (x', o'+e', e'), which (s, k)
// cells of the WFA recurrences can hold an offset at all does not depend on
// the sequences:
//
//   M_0[0] exists; I_s[k] exists if M_{s-o'-e'}[k-1] or I_{s-e'}[k-1] does;
//   D_s[k] exists if M_{s-o'-e'}[k+1] or D_{s-e'}[k+1] does; M_s[k] exists
//   if M_{s-x'}[k], I_s[k] or D_s[k] does.
//
// So the kernel is unrolled at compile time over exactly those cells (167
// M cells for steps 0..16 under (4, 6, 2), against 289 in the full
// triangle), every source index is a constant, the rows are plain
// registers, and a cell whose source cannot exist drops that candidate at
// compile time.  All lanes compute the same cells; each lane's own values
// differ.  The recurrences, the admissibility rule (a candidate offset c on
// diagonal k counts only if 0 <= c <= min(m, n + k), dropped before the
// maximum), the extension along matches, the termination test
// (M_s[m - n] == m) and the tie-break of the decision records are those of
// the short-pair kernel, so the results are bit-identical to it and to the
// oracle.
//
// LDS per wavefront, lane-interleaved (dword q of lane l at q * 64 + l, so
// 64 lanes reading "their" dword q hit 64 different banks): the pattern and
// the text in 2-bit little-endian words, and the bytes of one step's cells
// on their way to the history.  Per block: the (s, k) -> compact cell table
// and the (s, k) -> history byte table (the target test, the walk); the
// diagonal of each compact cell is a constant table read with scalar loads.
// Global memory per wavefront, lane-interleaved the same way (CIGAR mode):
// the history of every reachable M cell, its offset after extension (one
// byte, 0x80 for NULL; each step's staged dwords as they stand) and its
// 4-bit decision record (source of M: mismatch / end of insertion / end of
// deletion; whether I and D opened from M, packed in the cells' compile-time
// order), then a stage for the runs.  Keeping it out of LDS leaves room for four wavefronts per SIMD.
// The backtrace is the short kernel's walk, run by every lane on its own
// pair.
//
// A pair leaves through the overflow list (to the wider short-kernel passes
// and the general kernel) when a sequence is longer than LMAX bases, when
// its target diagonal lies outside the cells the kernel holds, when it needs
// more than CAP steps, or when its walk or runs do not fit.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "kernels.h"

namespace wfa {

namespace {

// NULL offset: far below every offset, and its low byte is 0x80, the NULL
// byte of the packed rows, the staging and the history
constexpr int LNUL = -(1 << 20) + 0x80;

// Which cells of steps 0..CAP can hold an offset (see above), and the
// compact history index of each reachable M cell.
template <int X, int OE, int E, int CAP, int KM>
struct LaneReach {
    static constexpr int W = 2 * KM + 1;
    bool m[CAP + 1][W] = {};
    bool i[CAP + 1][W] = {};
    bool d[CAP + 1][W] = {};
    short cidx[CAP + 1][W] = {};
    int ncells = 0;
    int kmax = 0;
    constexpr LaneReach() {
        for (int s = 0; s <= CAP; s++)
            for (int j = 0; j < W; j++) cidx[s][j] = -1;
        m[0][KM] = true;
        for (int s = 1; s <= CAP; s++) {
            for (int j = 0; j < W; j++) {
                bool iv = false, dv = false, mv = false;
                if (s >= OE && j >= 1 && m[s - OE][j - 1]) iv = true;
                if (s >= E && j >= 1 && i[s - E][j - 1]) iv = true;
                if (s >= OE && j + 1 < W && m[s - OE][j + 1]) dv = true;
                if (s >= E && j + 1 < W && d[s - E][j + 1]) dv = true;
                if (s >= X && m[s - X][j]) mv = true;
                i[s][j] = iv;
                d[s][j] = dv;
                m[s][j] = mv || iv || dv;
            }
        }
        int c = 0;
        for (int s = 0; s <= CAP; s++)
            for (int j = 0; j < W; j++)
                if (m[s][j]) {
                    cidx[s][j] = (short)c++;
                    const int k = j - KM;
                    kmax = (k > kmax) ? k : ((-k > kmax) ? -k : kmax);
                }
        ncells = c;
    }
};

template <class P>
__device__ __forceinline__ uint32_t lds_u32(P base, int dw) {
    return base[dw];
}

// 16 bases from base `pos` of a lane's sequence column (dword q at q * 64).
template <class P>
__device__ __forceinline__ uint32_t col_window16(P col, int pos) {
    const int q = pos >> 4;
    const uint32_t b = (uint32_t)(pos & 15) << 1;
    return __builtin_amdgcn_alignbit(col[q * 64 + 64], col[q * 64], b);
}

// 32 bases from base `pos` of a lane's sequence column (dword q at q * 64).
template <class P>
__device__ __forceinline__ uint64_t col_window32(P col, int pos) {
    const int q = pos >> 4;
    const uint32_t b = (uint32_t)(pos & 15) << 1;
    const uint32_t w0 = col[q * 64], w1 = col[q * 64 + 64], w2 = col[q * 64 + 128];
    const uint32_t lo = __builtin_amdgcn_alignbit(w1, w0, b);
    const uint32_t hi = __builtin_amdgcn_alignbit(w2, w1, b);
    return ((uint64_t)hi << 32) | lo;
}

template <class T>
using lptr = __attribute__((address_space(3))) T*;
template <class T>
using gptr_t = __attribute__((address_space(1))) T*;

template <int X, int OE, int E, int CAP, int LMAX, bool CIGAR>
struct LaneKernel {
    static constexpr int KM = CAP;  // array half-width; reachable |k| stays below it
    static constexpr int CAP1 = CAP + 1;
    using R = LaneReach<X, OE, E, CAP, KM>;
    static constexpr R reach{};
    static constexpr int W = R::W;
    static_assert(reach.kmax < KM, "reachable cells must stay inside the arrays");
    static constexpr int NC = reach.ncells;
    static constexpr int RM = (X > OE ? X : OE) + 1;  // ring of M rows (registers)
    static constexpr int RID = E + 1;                 // rings of I and D rows (registers)
    static constexpr int SQ = (LMAX >> 4) + 3;        // dwords per sequence column

    // the diagonal of each compact cell, as a constant table the extension
    // loop reads with scalar loads (its cell index is wave-uniform)
    struct Kof {
        int k[NC > 0 ? NC : 1] = {};
        constexpr Kof() {
            for (int s = 0; s <= CAP; s++)
                for (int j = 0; j < W; j++)
                    if (reach.cidx[s][j] >= 0) k[reach.cidx[s][j]] = j - KM;
        }
    };
    static constexpr Kof kof_tab{};

    static constexpr int first_cell(int s) {
        for (int j = 0; j < W; j++)
            if (reach.m[s][j]) return reach.cidx[s][j];
        return -1;
    }
    static constexpr int cells_of(int s) {
        int c = 0;
        for (int j = 0; j < W; j++) c += reach.m[s][j] ? 1 : 0;
        return c;
    }
    static constexpr int max_cells() {
        int mx = 0;
        for (int s = 0; s <= CAP; s++) mx = cells_of(s) > mx ? cells_of(s) : mx;
        return mx;
    }
    // A step's staged offsets, its M row words and its history words share
    // one layout: diagonal index J of step s at byte J - jbase(s), jbase(s)
    // the lowest reachable J rounded down to a multiple of four, so each
    // staged dword is a row word as it stands (bytes of unreachable diagonals
    // are never read).
    static constexpr int jlo(int s) {
        for (int j = 0; j < W; j++)
            if (reach.m[s][j]) return j;
        return -1;
    }
    static constexpr int jhi(int s) {
        for (int j = W - 1; j >= 0; j--)
            if (reach.m[s][j]) return j;
        return -1;
    }
    static constexpr int jbase(int s) { return jlo(s) < 0 ? 0 : (jlo(s) & ~3); }
    static constexpr int nwords(int s) { return jlo(s) < 0 ? 0 : (jhi(s) - jbase(s)) / 4 + 1; }
    static constexpr int hword(int s) {  // the history word of step s's first word
        int t = 0;
        for (int u = 0; u < s; u++) t += nwords(u);
        return t;
    }
    static constexpr int max_words() {
        int mx = 0;
        for (int s = 0; s <= CAP; s++) mx = nwords(s) > mx ? nwords(s) : mx;
        return mx;
    }
    // the history byte of each (s, k) cell (-1 where none), copied to LDS
    struct HistByte {
        short b[(CAP + 1) * W] = {};
        constexpr HistByte() {
            for (int s = 0; s <= CAP; s++)
                for (int j = 0; j < W; j++)
                    b[s * W + j] = reach.m[s][j] ? (short)(4 * hword(s) + j - jbase(s)) : (short)-1;
        }
    };
    static constexpr HistByte hist_byte{};
    // LDS per lane: both sequences and the staging bytes of one step's cells
    static constexpr int STW = max_words();
    static constexpr int LANE_DW = 2 * SQ + STW;
    static constexpr int WAVE_BYTES = LANE_DW * 64 * 4;
    // per block: the (s, k) -> compact cell table and the (s, k) -> history
    // byte table (int16 each), rounded to 256 bytes, so the lane columns that
    // follow sit at whole multiples of 64 dwords and paired column reads need
    // no base add
    static constexpr int TABLE_BYTES = (2 * (CAP + 1) * W * 2 + 255) & ~255;
    // CIGAR history per lane in global memory: the offset after extension of
    // every reachable cell (a byte; 0x80 NULL) in the staging layout, step
    // after step, then the cells' 4-bit decision records in compact order
    static constexpr int HMW = hword(CAP + 1);
    static constexpr int HRW = (NC + 7) / 8;
    static constexpr int HIST_DW = CIGAR ? HMW + HRW : 0;

    // Register rows hold one byte per diagonal, four diagonals to a word
    // (diagonal index J in byte J % 4 of word J / 4): every offset is at most
    // LMAX < 0x80, and 0x80 stands for NULL.  A row word is rebuilt at each
    // step from its reachable bytes only; bytes of unreachable diagonals are
    // never read.  A finished word passes through an empty asm, so the
    // compiler extracts each byte where a cell reads it instead of keeping
    // the unpacked bytes in registers.
    static constexpr int WP = (W + 3) / 4;
    struct St {
        uint32_t M[RM][WP];  // offsets after extension
        uint32_t I[RID][WP];
        uint32_t D[RID][WP];
        uint32_t pr;  // the record word being packed
    };
    template <int J>
    static __device__ __forceinline__ uint32_t byte_of(uint32_t w) {
        return (w >> (8 * (J & 3))) & 0xffu;
    }
    static constexpr bool reaches(int T, int S, int j) {
        return T == 0 ? reach.m[S][j] : (T == 1 ? reach.i[S][j] : reach.d[S][j]);
    }
    // whether J is the lowest / highest diagonal of its word that row type T
    // (0: M, 1: I, 2: D) reaches at step S
    static constexpr bool first_in_word(int T, int S, int J) {
        for (int j = J & ~3; j < J; j++)
            if (reaches(T, S, j)) return false;
        return true;
    }
    static constexpr bool last_in_word(int T, int S, int J) {
        for (int j = J + 1; j < ((J | 3) + 1) && j < W; j++)
            if (reaches(T, S, j)) return false;
        return true;
    }
    // byte J % 4 of w = the low byte of v (its other bytes are ignored): the
    // lowest reachable byte of a word starts it (bytes above it are left as
    // they come, and are either written next or never read), the others go
    // in by a byte permute that keeps the rest of the word
    template <int T, int S, int J>
    static __device__ __forceinline__ void put_byte(uint32_t& w, uint32_t v) {
        constexpr int p = J & 3;
        if constexpr (first_in_word(T, S, J)) {
            w = v << (8 * p);
        } else {
            constexpr uint32_t sel = (p == 0 ? 0x03020104u
                                      : p == 1 ? 0x03020400u : p == 2 ? 0x03040100u : 0x04020100u);
            w = __builtin_amdgcn_perm(v, w, sel);
        }
        if constexpr (last_in_word(T, S, J)) asm volatile("" : "+v"(w));
    }

    struct Lane {
        int n, m, kt;
        bool run;  // holds a pair that has not finished
        int S;
        lptr<uint32_t> P, T, G;  // sequence columns, staging column
        gptr_t<uint32_t> H;      // history column (global), dword d at H[d * 64]
    };

    static __device__ __forceinline__ lptr<uint8_t> gptr(const Lane& ln, int b) {
        return (lptr<uint8_t>)(ln.G + (b >> 2) * 64) + (b & 3);
    }

    // Phase 1 of a step, one cell: the recurrences from the register rows,
    // the decision record, and the offset before extension staged in LDS.
    template <int S, int J>
    static __device__ __forceinline__ void cell(St& st, Lane& ln) {
        if constexpr (reach.m[S][J]) {
            constexpr int k = J - KM;
            constexpr int g = J - jbase(S);  // staging byte
            const int L = min(ln.m, ln.n + k);  // largest admissible offset
            int Mv, Iv = LNUL, Dv = LNUL;
            [[maybe_unused]] uint32_t rec = 0;
            if constexpr (S == 0) {
                Mv = 0;
            } else {
                // candidates as unsigned distances t = L - c below the limit:
                // admissible offsets 0 <= t <= L, offsets past L negative
                // (huge); the largest admissible candidate is the smallest t,
                // floored at tn = L - NULL.  A source byte of 0x80 (NULL) is
                // past every limit, so it drops out.
                constexpr bool hA = S >= OE && J >= 1 && reach.m[S >= OE ? S - OE : 0][J >= 1 ? J - 1 : 0];
                constexpr bool hB = S >= E && J >= 1 && reach.i[S >= E ? S - E : 0][J >= 1 ? J - 1 : 0];
                constexpr bool hC = S >= OE && J + 1 < W && reach.m[S >= OE ? S - OE : 0][J + 1 < W ? J + 1 : 0];
                constexpr bool hE = S >= E && J + 1 < W && reach.d[S >= E ? S - E : 0][J + 1 < W ? J + 1 : 0];
                constexpr bool hX = S >= X && reach.m[S >= X ? S - X : 0][J];
                const uint32_t tn = (uint32_t)(L - LNUL);
                uint32_t ta = tn, tb = tn, tc = tn, te = tn, tx = tn;
                if constexpr (hA) ta = (uint32_t)(L - 1) - byte_of<J - 1>(st.M[(S - OE) % RM][(J - 1) / 4]);
                if constexpr (hB) tb = (uint32_t)(L - 1) - byte_of<J - 1>(st.I[(S - E) % RID][(J - 1) / 4]);
                if constexpr (hC) tc = (uint32_t)L - byte_of<J + 1>(st.M[(S - OE) % RM][(J + 1) / 4]);
                if constexpr (hE) te = (uint32_t)L - byte_of<J + 1>(st.D[(S - E) % RID][(J + 1) / 4]);
                if constexpr (hX) tx = (uint32_t)(L - 1) - byte_of<J>(st.M[(S - X) % RM][J / 4]);
                const uint32_t ti = min(min(ta, tb), tn);
                const uint32_t td = min(min(tc, te), tn);
                const uint32_t tm = min(min(tx, ti), td);
                Mv = L - (int)tm;
                Iv = L - (int)ti;
                Dv = L - (int)td;
                if constexpr (CIGAR) {
                    // tie-break: mismatch, then insertion, then deletion;
                    // gap open before gap extension
                    const uint32_t msrc = tx == tm ? 0u : (ti == tm ? 1u : 2u);
                    rec = msrc | (ta == ti ? 4u : 0u) | (tc == td ? 8u : 0u);
                    // materialise the record here: left to itself the compiler
                    // sinks these compares to the record word's store, keeping
                    // every candidate distance of eight cells live
                    asm volatile("" : "+v"(rec));
                }
            }
            // an offset is in [0, L] or exactly NULL (the minimum is floored
            // at tn), so its low byte is the offset or 0x80
            if constexpr (reach.i[S][J]) put_byte<1, S, J>(st.I[S % RID][J / 4], (uint32_t)Iv);
            if constexpr (reach.d[S][J]) put_byte<2, S, J>(st.D[S % RID][J / 4], (uint32_t)Dv);
            if constexpr (CIGAR) {
                constexpr int c = reach.cidx[S][J];
                if constexpr ((c & 7) == 0) st.pr = rec;
                else st.pr |= rec << (4 * (c & 7));
                if constexpr ((c & 7) == 7 || c == NC - 1) ln.H[(HMW + (c >> 3)) * 64] = st.pr;
            }
            // the low byte: the offset, or 0x80 for NULL
            *gptr(ln, g) = (uint8_t)Mv;
        }
    }

    // Phase 3 of a step, one staged dword (four diagonals): the offsets after
    // extension as they stand into the register row and (CIGAR) the history.
    template <int S, int Wi>
    static __device__ __forceinline__ void word_back(St& st, Lane& ln) {
        constexpr int rw = jbase(S) / 4 + Wi, hw = hword(S) + Wi;  // row word, history word
        const uint32_t w = ln.G[Wi * 64];
        st.M[S % RM][rw] = w;
        if constexpr (CIGAR) ln.H[hw * 64] = w;
    }

    template <int S, int... Js>
    static __device__ __forceinline__ void step_cells(St& st, Lane& ln,
                                                      std::integer_sequence<int, Js...>) {
        (cell<S, Js>(st, ln), ...);
    }
    template <int S, int... Ws>
    static __device__ __forceinline__ void step_back(St& st, Lane& ln,
                                                     std::integer_sequence<int, Ws...>) {
        (word_back<S, Ws>(st, ln), ...);
    }

    // Phase 2 of a step: extend every staged cell along matches, 32 bases
    // per compare (a wave-uniform loop; lanes with nothing to extend compare
    // at offset 0 and add nothing), stage the offset after extension, and
    // test the target cell.  One loop over the step's cells, unrolled by four
    // so the LDS reads of neighbouring cells overlap (5 M pairs at E = 4 %:
    // 1.79 against 1.84 ms per call rolled, with the packed rows); the target
    // test afterwards reads the one staged byte of the lane's target diagonal
    // through the (s, k) -> cell table.
    template <int S>
    static __device__ __forceinline__ bool extend_step(Lane& ln, lptr<const short> table) {
        constexpr int c0 = first_cell(S), ns = cells_of(S);
        bool term = false;
        if constexpr (ns > 0) {
#pragma unroll 4
            for (int j = 0; j < ns; j++) {
                const int k = kof_tab.k[c0 + j];
                constexpr int jb = jbase(S);
                lptr<uint8_t> bp = gptr(ln, k + KM - jb);
                const int Mv = *bp;  // 0x80 for NULL
                const int L = min(ln.m, ln.n + k);
                const bool go = ln.run && Mv < L;  // L <= LMAX < 0x80
                // a lane that does not extend keeps rem = 0, so it adds nothing
                // and its compares read its own or a neighbouring column of
                // this block's LDS (Mv - k within -16 .. 144), never stored
                int hp = Mv;
                int vp = Mv - k;
                int rem = go ? L - Mv : 0;
                // a 16-base compare first, for every cell (some lane of the
                // wave almost always extends, and testing for none costs more
                // than it saves); most cells stop within it, and the wave
                // runs on to 32-base compares only while a lane still matches
                uint32_t z16;
                asm("v_ffbl_b32 %0, %1" : "=v"(z16) : "v"(col_window16(ln.P, vp) ^ col_window16(ln.T, hp)));
                const int r16 = min((int)(min(z16, 32u) >> 1), rem);
                hp += r16;
                vp += r16;
                rem -= r16;
                bool more = __ballot(r16 == 16 && rem > 0) != 0;
                while (more) {
                    const uint64_t a = col_window32(ln.P, vp), bb = col_window32(ln.T, hp);
                    const uint64_t dx = a ^ bb;
                    // matching bases before the first mismatch: trailing zero
                    // bits of dx / 2, 32 when dx is 0 (v_ffbl gives ~0 for a zero
                    // word; the saturating add keeps it ~0 for the high word)
                    const uint32_t lo = (uint32_t)dx, hi = (uint32_t)(dx >> 32);
                    uint32_t zl, zh;
                    asm("v_ffbl_b32 %0, %1" : "=v"(zl) : "v"(lo));
                    asm("v_ffbl_b32 %0, %1" : "=v"(zh) : "v"(hi));
                    const int cp = (int)(min(min(zl, __builtin_elementwise_add_sat(zh, 32u)), 64u) >> 1);
                    const int r = min(cp, rem);
                    hp += r;
                    vp += r;
                    rem -= r;
                    // a lane that stopped short (a mismatch, or the end) compares
                    // at the same place again and adds 0 while others go on
                    more = __ballot(r == 32 && rem > 0) != 0;
                }
                if (go) *bp = (uint8_t)hp;
            }
            const int jt = ln.kt + KM;
            if (ln.run && jt >= 0 && jt < W) {
                const int c = table[S * W + jt];
                constexpr int jb = jbase(S);
                if (c >= 0) term = *gptr(ln, jt - jb) == ln.m;  // 0x80 (NULL) never equals m
            }
        }
        return term;
    }

    // The record word being packed when the forward pass stops after step
    // S (every lane finished): store it, so the walk never reads a stale word.
    template <int S>
    static __device__ __forceinline__ void flush(St& st, Lane& ln) {
        if constexpr (CIGAR && cells_of(S) > 0) {
            constexpr int last = first_cell(S) + cells_of(S) - 1;
            if constexpr ((last & 7) != 7 && last != NC - 1) ln.H[(HMW + (last >> 3)) * 64] = st.pr;
        }
    }

    // One score step; false once no lane of the wavefront is still running.
    template <int S>
    static __device__ __forceinline__ bool step(St& st, Lane& ln, lptr<const short> table) {
        // The lengths pass through an empty asm each step, so the per-diagonal
        // limits min(m, n + k) are recomputed (two instructions per cell)
        // instead of being kept in registers across the whole pass.
        // The history column's address passes through one too: otherwise the
        // compiler hoists the address of every history word out of the pair
        // loop and keeps them all in registers.
        asm volatile("" : "+v"(ln.n), "+v"(ln.m), "+v"(ln.H));
        step_cells<S>(st, ln, std::make_integer_sequence<int, W>{});
        const bool term = extend_step<S>(ln, table);
        step_back<S>(st, ln, std::make_integer_sequence<int, nwords(S)>{});
        const bool fin = ln.run && term;
        ln.S = fin ? S : ln.S;
        ln.run = ln.run && !term;
        if (__ballot(ln.run) == 0) {
            flush<S>(st, ln);
            return false;
        }
        return true;
    }

    template <int... Ss>
    static __device__ __forceinline__ void forward(St& st, Lane& ln, lptr<const short> table,
                                                   std::integer_sequence<int, Ss...>) {
        (step<Ss>(st, ln, table) && ...);  // stops after the step where every lane finished
    }
};

// At most 128 VGPRs (four wavefronts per SIMD).  With the register rows as
// packed bytes the 16-step CIGAR form needs 125 and no scratch (with the
// extension loop unrolled by four and the row words taken from the staged
// dwords as they stand): a 5 M-pair call
// at E = 4 % took 1.87 ms (rolled) against 2.02 ms with one register per
// diagonal (128 VGPRs and 48 dwords per lane in scratch), and 1.88 ms at five
// wavefronts (96 VGPRs, 30 spilled), in alternating runs on one device.
template <int X, int OE, int E, int CAP, int LMAX, bool CIGAR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_lane(LaneArgs a,
                                                                                    int persistent) {
    using K = LaneKernel<X, OE, E, CAP, LMAX, CIGAR>;
    extern __shared__ __align__(16) unsigned char lds[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    lptr<unsigned char> ldsb = (lptr<unsigned char>)lds;
    // per block: the (s, k) -> compact cell table, the (s, k) -> history byte
    // table, then one region per wavefront
    lptr<short> table = (lptr<short>)ldsb;
    lptr<short> hbt = table + K::CAP1 * K::W;
    for (int i = threadIdx.x; i < (K::CAP1) * K::W; i += blockDim.x) {
        const int s = i / K::W, j = i % K::W;
        table[i] = (short)K::reach.cidx[s][j];
        hbt[i] = K::hist_byte.b[i];
    }
    __syncthreads();
    lptr<uint32_t> wbase = (lptr<uint32_t>)(ldsb + K::TABLE_BYTES + wave * K::WAVE_BYTES) + lane;
    typename K::Lane ln;
    ln.P = wbase;
    ln.T = wbase + K::SQ * 64;
    ln.G = wbase + 2 * K::SQ * 64;
    // this wavefront's history and run-stage region (HIST_DW + slot_cap rows
    // of 64 dwords; one region per launched wavefront)
    ln.H = (gptr_t<uint32_t>)a.hist +
           ((uint64_t)(blockIdx.x * wpb + wave) * (CIGAR ? K::HIST_DW + a.slot_cap : 0)) * 64 + lane;
    // persistent: LANE_QUEUES counters (one per 128-byte line), wavefront w
    // drawing from counter w % LANE_QUEUES; the i-th claim from counter q is
    // the group of 64 queue entries number i * LANE_QUEUES + q, so every
    // counter serves an interleaved share of the queue (of the same mix of
    // costs) and no single address takes every wavefront's atomics
    const uint32_t qid = (blockIdx.x * wpb + wave) % LANE_QUEUES;
    for (uint32_t iter = 0;; iter++) {
        uint32_t qbase;
        if (persistent) {
            uint32_t t = 0;
            if (lane == 0) t = atomicAdd(a.queue + qid * 32, 1u);
            const uint32_t i = __builtin_amdgcn_readfirstlane(t);
            const uint64_t g = (uint64_t)i * LANE_QUEUES + qid;
            qbase = g * 64 >= a.num ? a.num : (uint32_t)(g * 64);
        } else {
            if (iter) break;
            qbase = (blockIdx.x * wpb + wave) * 64;
        }
        if (qbase >= a.num) break;
        const uint32_t q = qbase + lane;
        uint32_t pair = 0;
        bool active = q < a.num;
        if (active) {
            pair = a.order ? a.order[q] : q;
            if (pair >= a.npairs) {  // a corrupt permutation must not fault: skip the entry
                active = false;
                pair = 0;
            }
        }
        int n = 0, m = 0;
        uint64_t ps = 0, ts = 0;
        if (active) {
            const PairDesc d = a.pairs[pair];
            n = (int)d.p_len;
            m = (int)d.t_len;
            ps = d.p_start;
            ts = d.t_start;
        }
        ln.n = n;
        ln.m = m;
        ln.kt = m - n;
        // pairs this kernel cannot hold leave at once
        bool fits = n <= LMAX && m <= LMAX && ln.kt >= -K::reach.kmax && ln.kt <= K::reach.kmax;
        ln.run = active && fits;
        ln.S = -1;
        // stage both sequences in the lane's columns (zero past their ends)
        {
            const int nwp = ln.run ? (n + 31) >> 5 : 0, nwt = ln.run ? (m + 31) >> 5 : 0;
#pragma unroll
            for (int w = 0; w < (K::SQ + 1) / 2; w++) {
                const uint64_t pv = w < nwp ? a.pw[ps + w] : 0ull;
                const uint64_t tv = w < nwt ? a.tw[ts + w] : 0ull;
                if (2 * w < K::SQ) {
                    ln.P[(2 * w) * 64] = (uint32_t)pv;
                    ln.T[(2 * w) * 64] = (uint32_t)tv;
                }
                if (2 * w + 1 < K::SQ) {
                    ln.P[(2 * w + 1) * 64] = (uint32_t)(pv >> 32);
                    ln.T[(2 * w + 1) * 64] = (uint32_t)(tv >> 32);
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        typename K::St st;
        if (__ballot(ln.run) != 0)
            K::forward(st, ln, (lptr<const short>)table, std::make_integer_sequence<int, CAP + 1>{});
        // lanes still running after CAP steps leave through the overflow list
        bool overflow = active && ln.S < 0;
        int nr = 0;
        if (CIGAR && active && !overflow) {
            // The short kernel's walk, on this lane's pair: one event per
            // iteration -- at M cell (s, k) the record names the source (a
            // mismatch from M at s - x, or the end of a gap whose chain of I
            // or D cells is followed back to the M cell it opened from); the
            // iteration emits the cell's match run and the event's edit run
            // (extending the open run when nothing matched in between and
            // the op is the same) and moves to the source M cell.  Runs go
            // to the pair's slot last to first.
            const int cap_runs = a.slot_cap;
            // runs are staged lane-interleaved after the wavefront's history
            // (run r of this lane at stage[r * 64]), so every store of the
            // walk writes one contiguous 256-byte row
            gptr_t<uint32_t> slot = ln.H + K::HIST_DW * 64;
            auto cidx = [&](int s, int k) -> int {
                if (s < 0 || s > CAP || k < -K::KM || k > K::KM) return -1;
                return table[s * K::W + k + K::KM];
            };
            // the offset of a reachable cell (s, k): byte hbt of the history
            auto hm = [&](int s, int k) -> int {
                const int hb = hbt[s * K::W + k + K::KM];
                const uint32_t w = ln.H[(hb >> 2) * 64];
                const int b = (int)((w >> (8 * (hb & 3))) & 0xFFu);
                return b & 0x80 ? -1 : b;
            };
            auto hr = [&](int c) -> int {
                const uint32_t w = ln.H[(K::HMW + (c >> 3)) * 64];
                return (int)((w >> (4 * (c & 7))) & 15u);
            };
            int cop = -1, clen = 0;
            int s = ln.S, k = ln.kt, h = m;
            bool bad = false;
            for (;;) {
                const int c = cidx(s, k);
                if (c < 0) {
                    bad = true;
                    break;
                }
                int h0 = 0, hn = 0, L = 1, op = 0, s2 = 0, dk = 0;
                if (s > 0) {
                    const int f = hr(c);
                    const int ms = f & 3;
                    if (ms == 0) {
                        const int cs = cidx(s - X, k);
                        if (cs < 0) {
                            bad = true;
                            break;
                        }
                        hn = hm(s - X, k);
                        h0 = hn + 1;
                        s2 = s - X;
                    } else {
                        const int bit = ms == 1 ? 4 : 8;
                        const int dj = ms == 1 ? -1 : 1;
                        int sc = s, kc = k, fc = f;
                        while (!(fc & bit)) {  // still extending: one step back
                            sc -= E;
                            kc += dj;
                            const int cc = cidx(sc, kc);
                            if (sc <= 0 || cc < 0) break;
                            L++;
                            fc = hr(cc);
                        }
                        const int co = cidx(sc - OE, kc + dj);
                        if (!(fc & bit) || co < 0) {
                            bad = true;  // a gap with no opening: inconsistent
                            break;
                        }
                        hn = hm(sc - OE, kc + dj);
                        h0 = ms == 1 ? hn + L : hn;  // insertions consume text
                        s2 = sc - OE;
                        dk = dj * L;
                    }
                    op = ms + 1;  // op codes: X=1 I=2 D=3
                }
                const bool last = s == 0;
                const int mlen = h - h0;
                if (mlen < 0 || hn < 0) {
                    bad = true;
                    break;
                }
                const bool hasM = mlen > 0;
                const bool flushr = cop >= 0 && (hasM || last || cop != op);
                if (flushr) {
                    if (nr < cap_runs) slot[nr * 64] = ((uint32_t)clen << 4) | (uint32_t)cop;
                    nr++;
                }
                if (hasM) {
                    if (nr < cap_runs) slot[nr * 64] = ((uint32_t)mlen << 4);
                    nr++;
                }
                if (last) break;
                clen = (flushr || hasM) ? L : clen + L;
                cop = op;
                s = s2;
                k += dk;
                h = hn;
            }
            if (bad || nr > cap_runs) overflow = true;
        }
        // CIGAR: the 64 pairs' runs packed one after another at the start of
        // the group's slot area (64 * slot_cap words from queue position
        // qbase on), so the compaction reads dense data
        uint64_t src = 0;
        if (CIGAR) {
            const int cnt = (active && !overflow) ? nr : 0;
            int incl = cnt;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(incl, off);
                incl += lane >= off ? t : 0;
            }
            src = (uint64_t)qbase * a.slot_cap + (uint64_t)(incl - cnt);
            const gptr_t<uint32_t> stage = ln.H + K::HIST_DW * 64;
            for (int r = 0; r < cnt; r++) a.slots[src + r] = stage[r * 64];
        }
        if (active) {
            if (overflow) {
                const uint32_t at = atomicAdd(a.ovf_count, 1u);
                a.ovf_list[at] = pair;
            } else {
                a.scores[pair] = ln.S * a.pen.g;
                a.nruns[pair] = CIGAR ? (uint32_t)nr : 0u;
                if (CIGAR) a.run_src[pair] = src;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

template <int X, int OE, int E, int CAP, int LMAX>
struct LaneShape {
    static int lds_bytes(bool cigar, int waves) {
        return cigar ? LaneKernel<X, OE, E, CAP, LMAX, true>::TABLE_BYTES +
                           waves * LaneKernel<X, OE, E, CAP, LMAX, true>::WAVE_BYTES
                     : LaneKernel<X, OE, E, CAP, LMAX, false>::TABLE_BYTES +
                           waves * LaneKernel<X, OE, E, CAP, LMAX, false>::WAVE_BYTES;
    }
    // history and run stage of one wavefront (slot_cap runs per lane)
    static int hist_dwords(bool cigar, int slot_cap) {
        return cigar ? (LaneKernel<X, OE, E, CAP, LMAX, true>::HIST_DW + slot_cap) * 64 : 0;
    }
    static hipError_t launch(const LaneArgs& a, bool cigar, bool persistent, int bt, int grid,
                             hipStream_t s) {
        const int lds = lds_bytes(cigar, bt / 64);
        if (cigar)
            hipLaunchKernelGGL((k_lane<X, OE, E, CAP, LMAX, true>), dim3(grid), dim3(bt), lds, s, a,
                               persistent ? 1 : 0);
        else
            hipLaunchKernelGGL((k_lane<X, OE, E, CAP, LMAX, false>), dim3(grid), dim3(bt), lds, s, a,
                               persistent ? 1 : 0);
        return hipGetLastError();
    }
    static int occupancy(bool cigar, int bt) {
        int blocks = 0;
        const int lds = lds_bytes(cigar, bt / 64);
        const hipError_t e =
            cigar ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                        &blocks, (const void*)k_lane<X, OE, E, CAP, LMAX, true>, bt, lds)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                        &blocks, (const void*)k_lane<X, OE, E, CAP, LMAX, false>, bt, lds);
        return e == hipSuccess ? blocks : 0;
    }
    static int kmax() { return LaneKernel<X, OE, E, CAP, LMAX, false>::reach.kmax; }
};

// Shapes built: scaled penalties (2, 4, 1) -- x = 4, o = 6, e = 2 and their
// multiples -- with 8 or 16 score steps, sequences up to 127 bases.
#define WFA_LANE_SHAPES(F) \
    F(2, 4, 1, 8, 127)     \
    F(2, 4, 1, 16, 127)

}  // namespace

bool lane_supported(const Pen& pen, int cap, uint32_t max_len) {
#define WFA_LANE_CASE(PX, POE, PE, PC, PLM) \
    if (pen.x == PX && pen.oe == POE && pen.e == PE && cap == PC && max_len <= (uint32_t)PLM) return true;
    WFA_LANE_SHAPES(WFA_LANE_CASE)
#undef WFA_LANE_CASE
    return false;
}

int lane_kmax(const Pen& pen, int cap) {
#define WFA_LANE_CASE(PX, POE, PE, PC, PLM) \
    if (pen.x == PX && pen.oe == POE && pen.e == PE && cap == PC) return LaneShape<PX, POE, PE, PC, PLM>::kmax();
    WFA_LANE_SHAPES(WFA_LANE_CASE)
#undef WFA_LANE_CASE
    return -1;
}

int lane_lds_bytes(const Pen& pen, int cap, bool cigar, int block_threads) {
#define WFA_LANE_CASE(PX, POE, PE, PC, PLM) \
    if (pen.x == PX && pen.oe == POE && pen.e == PE && cap == PC) \
        return LaneShape<PX, POE, PE, PC, PLM>::lds_bytes(cigar, block_threads / 64);
    WFA_LANE_SHAPES(WFA_LANE_CASE)
#undef WFA_LANE_CASE
    return -1;
}

size_t lane_hist_bytes_per_wave(const Pen& pen, int cap, bool cigar, int slot_cap) {
#define WFA_LANE_CASE(PX, POE, PE, PC, PLM) \
    if (pen.x == PX && pen.oe == POE && pen.e == PE && cap == PC) \
        return (size_t)LaneShape<PX, POE, PE, PC, PLM>::hist_dwords(cigar, slot_cap) * 4;
    WFA_LANE_SHAPES(WFA_LANE_CASE)
#undef WFA_LANE_CASE
    return 0;
}

int lane_max_blocks_per_cu(const Pen& pen, int cap, bool cigar, int block_threads) {
#define WFA_LANE_CASE(PX, POE, PE, PC, PLM) \
    if (pen.x == PX && pen.oe == POE && pen.e == PE && cap == PC) \
        return LaneShape<PX, POE, PE, PC, PLM>::occupancy(cigar, block_threads);
    WFA_LANE_SHAPES(WFA_LANE_CASE)
#undef WFA_LANE_CASE
    return 0;
}

hipError_t launch_lane(const LaneArgs& a, int cap, bool cigar, bool persistent, int block_threads,
                       int grid, hipStream_t s) {
#define WFA_LANE_CASE(PX, POE, PE, PC, PLM) \
    if (a.pen.x == PX && a.pen.oe == POE && a.pen.e == PE && cap == PC) \
        return LaneShape<PX, POE, PE, PC, PLM>::launch(a, cigar, persistent, block_threads, grid, s);
    WFA_LANE_SHAPES(WFA_LANE_CASE)
#undef WFA_LANE_CASE
    return hipErrorInvalidValue;
}

}  // namespace wfa
