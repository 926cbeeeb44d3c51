// C-ABI of the batched WFA library: validation, planning, device workspace
// and the launch sequence of one batch.  All alignment arithmetic runs in the
// HIP kernels (kernels.hip); this file only moves data and decides which
// kernel gets which pairs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/wfa.h"
#include "kernels.h"
#include "internal.h"

using namespace wfa;

namespace {

int gcd3(int a, int b, int c) { return std::gcd(std::gcd(a, b), c); }

double elapsed_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return (double)ms;
}

}  // namespace

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
void Workspace::use_fixed(void* base, size_t size) {
    for (Buf* b : all()) *b = Buf{};
    fixed_base = (unsigned char*)base;
    fixed_size = size;
    fixed_top = 0;
    total = 0;
    budget = size;
    generation++;
}

int Workspace::ensure(Buf& b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~(size_t)255;
    if (b.bytes >= bytes) return WFA_OK;
    release(b);
    generation++;
    if (fixed_base) {  // carve from the region (256-byte aligned like its base)
        if (fixed_top + bytes > fixed_size) return WFA_E_NOMEM;
        b.ptr = fixed_base + fixed_top;
        b.bytes = bytes;
        fixed_top += bytes;
        total = fixed_top;
        return WFA_OK;
    }
    if (total + bytes > budget) return WFA_E_NOMEM;
    // stream-ordered on the engine's stream, which is then drained so the
    // block is ready for any stream (a plain hipMalloc / hipFree would
    // synchronise the whole device, stalling every other engine)
    const hipError_t he = own[0] ? hipMallocAsync(&b.ptr, bytes, own[0]) : hipMalloc(&b.ptr, bytes);
    if (he != hipSuccess || (own[0] && hipStreamSynchronize(own[0]) != hipSuccess)) {
        (void)hipGetLastError();
        if (he == hipSuccess && b.ptr) (void)hipFree(b.ptr);
        b.ptr = nullptr;
        return WFA_E_NOMEM;
    }
    b.bytes = bytes;
    total += bytes;
    return WFA_OK;
}

int Workspace::grow_keep(Buf& b, size_t bytes, size_t keep, hipStream_t s) {
    if (b.bytes >= bytes) return WFA_OK;
    Buf nb;
    int rc = ensure(nb, std::max(bytes, b.bytes * 2));
    if (rc != WFA_OK) rc = ensure(nb, bytes);
    if (rc != WFA_OK) return rc;
    if ((keep && hipMemcpyAsync(nb.ptr, b.ptr, keep, hipMemcpyDeviceToDevice, s) != hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        release(nb);
        return WFA_E_DEVICE;
    }
    release(b);
    b = nb;
    return WFA_OK;
}

void Workspace::release(Buf& b) {
    if (fixed_base) {
        if (b.ptr && (unsigned char*)b.ptr + b.bytes == fixed_base + fixed_top) fixed_top -= b.bytes;
        total = fixed_top;
        b = Buf{};
        return;
    }
    if (b.ptr) {
        if (own[0]) {
            // nothing of this engine may still use the block
            for (hipStream_t q : own)
                if (q) (void)hipStreamSynchronize(q);
            if (hipFreeAsync(b.ptr, own[0]) != hipSuccess || hipStreamSynchronize(own[0]) != hipSuccess)
                (void)hipGetLastError();
        } else {
            (void)hipFree(b.ptr);
        }
        total -= b.bytes;
    }
    b.ptr = nullptr;
    b.bytes = 0;
}

void Workspace::release_all() {
    if (fixed_base) {
        use_fixed(fixed_base, fixed_size);
        return;
    }
    for (Buf* b : all()) release(*b);
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
    pinned_bytes = 0;
}

int Workspace::ensure_pinned(size_t bytes) {
    if (pinned_bytes >= bytes) return WFA_OK;
    if (fixed_base) return WFA_E_NOMEM;  // never allocates
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
    pinned_bytes = 0;
    if (hipHostMalloc(&pinned, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        pinned = nullptr;
        return WFA_E_NOMEM;
    }
    pinned_bytes = bytes;
    return WFA_OK;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
int engine_init(Engine* e, int device, size_t budget) {
    int ndev = 0;
    hipError_t he = hipGetDeviceCount(&ndev);
    if (he != hipSuccess || device < 0 || device >= ndev) {
        if (std::getenv("WFA_DEBUG"))
            std::fprintf(stderr, "libwfa: hipGetDeviceCount -> %s, %d devices\n",
                         hipGetErrorString(he), ndev);
        (void)hipGetLastError();
        return WFA_E_DEVICE;
    }
    he = hipSetDevice(device);
    if (he != hipSuccess) {
        std::fprintf(stderr, "libwfa: hipSetDevice -> %s\n", hipGetErrorString(he));
        return WFA_E_DEVICE;
    }
    e->device = device;
    // default budget: three quarters of the device's memory (the workspace
    // grows only as far as the batches need)
    size_t total_mem = 0;
    {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, device) == hipSuccess) total_mem = p.totalGlobalMem;
        else (void)hipGetLastError();
    }
    e->ws.budget = budget ? budget : (total_mem ? total_mem / 4 * 3 : ((size_t)64 << 30));
    he = hipHostMalloc(&e->readback, 256, hipHostMallocDefault);
    if (he != hipSuccess) {
        std::fprintf(stderr, "libwfa: hipHostMalloc -> %s\n", hipGetErrorString(he));
        e->readback = nullptr;
        return WFA_E_DEVICE;
    }
    // default priority: every stream of the library runs at the same priority
    he = hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking);
    if (he != hipSuccess) {
        std::fprintf(stderr, "libwfa: hipStreamCreate -> %s\n", hipGetErrorString(he));
        e->stream = nullptr;
        return WFA_E_DEVICE;
    }
    if (hipStreamCreateWithFlags(&e->h2d, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&e->d2h, hipStreamNonBlocking) != hipSuccess) {
        std::fprintf(stderr, "libwfa: hipStreamCreate (copy streams) failed\n");
        (void)hipGetLastError();
        return WFA_E_DEVICE;
    }
    e->ws.own[0] = e->stream;
    e->ws.own[1] = e->h2d;
    e->ws.own[2] = e->d2h;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) e->num_cus = prop.multiProcessorCount;
    if (e->num_cus <= 0) e->num_cus = 256;
    for (auto& ev : e->ev) (void)hipEventCreate(&ev);
    std::memset(&e->opt, 0, sizeof(e->opt));
    std::memset(&e->last, 0, sizeof(e->last));
    return WFA_OK;
}

void engine_destroy(Engine* e) {
    (void)hipSetDevice(e->device);
    if (e->stream) (void)hipStreamSynchronize(e->stream);
    graph_cache_clear(e);
    e->ws.release_all();
    for (auto& ev : e->ev)
        if (ev) (void)hipEventDestroy(ev);
    if (e->readback) (void)hipHostFree(e->readback);
    e->readback = nullptr;
    if (e->stream) (void)hipStreamDestroy(e->stream);
    if (e->h2d) (void)hipStreamDestroy(e->h2d);
    if (e->d2h) (void)hipStreamDestroy(e->d2h);
    e->stream = e->h2d = e->d2h = nullptr;
}

extern "C" int wfa_ctx_create(int device, size_t hbm_budget_bytes, wfa_ctx** out) {
    if (!out) return WFA_E_INVAL;
    *out = nullptr;
    wfa_ctx* c = new wfa_ctx();
    int rc = engine_init(c, device, hbm_budget_bytes);
    // set-up of the allocation-free entry point: the scratch array's address
    // on this device, and an engine (streams, events) whose workspace is
    // carved from it
    if (rc == WFA_OK) rc = noalloc_setup(device);
    if (rc == WFA_OK) {
        c->fixed.reset(new Engine());
        rc = engine_init(c->fixed.get(), device, noalloc_scratch_bytes());
        if (rc == WFA_OK) c->fixed->ws.use_fixed(noalloc_scratch(device), noalloc_scratch_bytes());
    }
    if (rc != WFA_OK) {
        if (c->fixed) engine_destroy(c->fixed.get());
        engine_destroy(c);
        delete c;
        return rc;
    }
    *out = c;
    return WFA_OK;
}

extern "C" void wfa_ctx_destroy(wfa_ctx* ctx) {
    if (!ctx) return;
    for (auto& e : ctx->idle)
        if (e) engine_destroy(e.get());
    ctx->idle.clear();
    if (ctx->fixed) engine_destroy(ctx->fixed.get());  // the scratch array itself stays
    ctx->fixed.reset();
    engine_destroy(ctx);
    delete ctx;
}

extern "C" int wfa_set_options(wfa_ctx* ctx, const wfa_options* opt) {
    if (!ctx) return WFA_E_INVAL;
    if (!opt) {
        std::memset(&ctx->opt, 0, sizeof(ctx->opt));
        return WFA_OK;
    }
    if (opt->schedule < 0 || opt->schedule > WFA_SCHED_GENERAL) return WFA_E_INVAL;
    if (opt->window && opt->window != 16 && opt->window != 24 && opt->window != 32 &&
        opt->window != 48 && opt->window != 64 && opt->window != 128 && opt->window != 256)
        return WFA_E_INVAL;
    if (opt->lanes_per_pair && opt->lanes_per_pair != 8 && opt->lanes_per_pair != 16 &&
        opt->lanes_per_pair != 32 && opt->lanes_per_pair != 64)
        return WFA_E_INVAL;
    if (opt->window && opt->lanes_per_pair && !short_shape_supported(opt->window, opt->lanes_per_pair))
        return WFA_E_INVAL;
    if (opt->step_cap < 0 || opt->step_cap > 4096) return WFA_E_INVAL;
    if (opt->block_threads && (opt->block_threads < 64 || opt->block_threads > 256 ||
                               opt->block_threads % 64))
        return WFA_E_INVAL;
    if (opt->general_pairs < 0) return WFA_E_INVAL;
    if (opt->use_graph < -1 || opt->use_graph > 2) return WFA_E_INVAL;
    if (opt->bucket < -1 || opt->bucket > 1) return WFA_E_INVAL;
    if (opt->general_slice_kib < 0 || opt->general_slice_kib > (1 << 22)) return WFA_E_INVAL;
    if (opt->general_step_limit < 0) return WFA_E_INVAL;
    if (opt->general_checkpoint < -1 || opt->general_checkpoint > GENERAL_CKPT_MAX)
        return WFA_E_INVAL;
    if (opt->lane_kernel < -1 || opt->lane_kernel > 1) return WFA_E_INVAL;
    if (opt->host_chunk_pairs < 0) return WFA_E_INVAL;
    if (opt->cascade_window < -1 ||
        (opt->cascade_window > 0 &&
         !short_shape_supported(opt->cascade_window, default_lanes(opt->cascade_window))))
        return WFA_E_INVAL;
    ctx->opt = *opt;
    return WFA_OK;
}

extern "C" int wfa_set_ends_free(wfa_ctx* ctx, const wfa_ends_free* ends) {
    if (!ctx) return WFA_E_INVAL;
    if (!ends) {
        ctx->ends = Ends{0, 0, 0, 0};
        return WFA_OK;
    }
    if (ends->pattern_begin_free > WFA_MAX_LENGTH || ends->pattern_end_free > WFA_MAX_LENGTH ||
        ends->text_begin_free > WFA_MAX_LENGTH || ends->text_end_free > WFA_MAX_LENGTH)
        return WFA_E_INVAL;
    const bool free_ends = ends->pattern_begin_free || ends->pattern_end_free ||
                           ends->text_begin_free || ends->text_end_free;
    if (free_ends && ctx->heur.mwl > 0) return WFA_E_INVAL;  // the heuristic is global-only
    ctx->ends = Ends{(int)ends->pattern_begin_free, (int)ends->pattern_end_free,
                     (int)ends->text_begin_free, (int)ends->text_end_free};
    return WFA_OK;
}

extern "C" int wfa_set_heuristic(wfa_ctx* ctx, const wfa_heuristic* h) {
    if (!ctx) return WFA_E_INVAL;
    if (!h || h->min_wavefront_length == 0) {
        if (h && h->max_distance_threshold < 0) return WFA_E_INVAL;
        ctx->heur = Heuristic{0, 0};
        return WFA_OK;
    }
    if (h->min_wavefront_length < 0 || h->max_distance_threshold < 0) return WFA_E_INVAL;
    if (ctx->ends.pb || ctx->ends.pe || ctx->ends.tb || ctx->ends.te) return WFA_E_INVAL;
    ctx->heur = Heuristic{h->min_wavefront_length, h->max_distance_threshold};
    return WFA_OK;
}

extern "C" int wfa_last_stats(const wfa_ctx* ctx, wfa_stats* out) {
    if (!ctx || !out) return WFA_E_INVAL;
    *out = ctx->last;
    return WFA_OK;
}

extern "C" const char* wfa_strerror(int status) {
    switch (status) {
    case WFA_OK: return "ok";
    case WFA_E_INVAL: return "invalid argument";
    case WFA_E_ALPHABET: return "sequence byte outside ACGTacgt";
    case WFA_E_NOMEM: return "HBM budget or device memory exhausted";
    case WFA_E_CAPACITY: return "CIGAR buffer too small (see cigar_needed)";
    case WFA_E_DEVICE: return "HIP runtime error";
    case WFA_E_TOO_LONG: return "sequence longer than WFA_MAX_LENGTH";
    case WFA_E_BUSY: return "not finished / queue full";
    case WFA_E_NOTFOUND: return "unknown ticket";
    case WFA_E_LIMIT: return "the general kernel gave up on a pair (step limit or internal error)";
    default: return "unknown status";
    }
}

// ---------------------------------------------------------------------------
// planning helpers
// ---------------------------------------------------------------------------
int make_pen(const wfa_penalties& p, Pen* out) {
    if (p.mismatch <= 0 || p.gap_extend <= 0 || p.gap_open < 0) return WFA_E_INVAL;
    if (p.mismatch > (1 << 20) || p.gap_open > (1 << 20) || p.gap_extend > (1 << 20))
        return WFA_E_INVAL;
    const int g = gcd3(p.mismatch, p.gap_open, p.gap_extend);
    out->g = g;
    out->x = p.mismatch / g;
    out->oe = (p.gap_open + p.gap_extend) / g;
    out->e = p.gap_extend / g;
    out->pre = std::max(out->x, std::max(out->oe, out->e));
    if (out->pre + 1 > GENERAL_MAX_RING) return WFA_E_INVAL;
    return WFA_OK;
}

// Steps a window of W diagonals can run before the wavefront can reach its
// edge: a gap must open (oe steps) and then spread W/2 diagonals (e steps
// each); a mismatch step beyond that adds nothing that stays in the window.
int default_cap(const Pen& pen, int window) { return pen.oe + (window / 2) * pen.e + pen.x; }

// Several diagonals per lane by default: outer layers are computed only once
// the wavefront reaches them, so narrow score steps cost one layer; windows
// up to 32 use 8-lane groups (8 pairs per wavefront).
int default_lanes(int window) {
    if (window <= 32) return 8;
    return window >= 128 ? 64 : window / 2;
}

int short_plan(Engine* ctx, const Pen& pen, bool cigar, int window, int lanes, int cap,
               uint32_t max_len, ShortPlan* sp) {
    if (!short_shape_supported(window, lanes)) return WFA_E_INVAL;
    sp->window = window;
    sp->lanes = lanes;
    sp->cap = cap;
    sp->seq_words = (int)((max_len + 31) / 32) + 1;
    // offsets: I and D rows in rings of e + 1 (a step reads them back e
    // steps); M rows in a ring of pre + 1 in score mode, all of them (after
    // one NULL row) in CIGAR mode, which adds a 4-bit decision record per
    // cell and step for the backtrace
    sp->ring = cigar ? cap + 2 : pen.pre + 1;
    sp->ring2 = pen.e + 1;
    // int8 offsets hold lengths up to 127; a NULL (-128) drifts up by at most
    // one per step, so it stays negative for caps below 100
    sp->row_bytes = (max_len <= 127 && cap < 100) ? 1 : 2;
    const int RW = window + 2;
    // runs: every non-match op costs at least min(x, e) (in units of g)
    const int minc = std::min(pen.x, pen.e);
    sp->slot_cap = 2 * ((cap / minc) + 1) + 2;
    // ends-free: a free prefix and a free suffix run
    if (ctx->ends.pb || ctx->ends.pe || ctx->ends.tb || ctx->ends.te) sp->slot_cap += 2;
    // the I/D rings are free during the backtrace, which stages the runs
    // there (two spare words take the stores of a walk that overflows)
    sp->id_off = (sp->ring * RW * sp->row_bytes + 15) & ~15;
    const int id_bytes =
        std::max(2 * sp->ring2 * RW * sp->row_bytes, cigar ? 4 * (sp->slot_cap + 2) : 0);
    sp->rows_bytes = (sp->id_off + id_bytes + 15) & ~15;
    const int rec_bytes = cigar ? (((cap + 1) * (window / 2)) + 15) & ~15 : 0;
    sp->group_bytes = sp->rows_bytes + rec_bytes + 2 * sp->seq_words * 8;
    sp->group_bytes = (sp->group_bytes + 15) & ~15;
    int bt = ctx->opt.block_threads ? ctx->opt.block_threads : 256;
    while (bt > 64 && (size_t)short_groups_per_block(lanes, bt) * sp->group_bytes > 64 * 1024)
        bt -= 64;
    if ((size_t)short_groups_per_block(lanes, bt) * sp->group_bytes > 64 * 1024) return WFA_E_NOMEM;
    sp->block_threads = bt;
    sp->lds_per_block = short_groups_per_block(lanes, bt) * sp->group_bytes;
    return WFA_OK;
}

// ---------------------------------------------------------------------------
// batch entry points
// ---------------------------------------------------------------------------
extern "C" int wfa_align_batch(wfa_ctx* ctx, const void* patterns, const void* texts,
                               const wfa_pair* pairs, size_t num_pairs, wfa_encoding enc,
                               wfa_memspace mem, wfa_penalties pen, wfa_mode mode, int32_t* scores,
                               uint32_t* cigar_runs, size_t cigar_capacity,
                               uint64_t* cigar_offsets, size_t* cigar_needed, int64_t* bad_pair,
                               void* stream) {
    if (bad_pair) *bad_pair = -1;
    if (!ctx) return WFA_E_INVAL;
    BatchIO io{patterns, texts, pairs, num_pairs, enc, mem, pen, mode,
               scores, cigar_runs, cigar_capacity, cigar_offsets};
    return engine_align(ctx, io, (hipStream_t)stream, cigar_needed, bad_pair);
}

#define API_HIPCHK(x)                \
    do {                             \
        if ((x) != hipSuccess) {     \
            (void)hipGetLastError(); \
            return WFA_E_DEVICE;     \
        }                            \
    } while (0)

extern "C" int wfa_copy_last_cigars(wfa_ctx* ctx, uint32_t* runs, size_t capacity,
                                    uint64_t* offsets) {
    if (!ctx || !ctx->last_valid) return WFA_E_INVAL;
    if (capacity < ctx->last_total) return WFA_E_CAPACITY;
    if (ctx->last_total && !runs) return WFA_E_INVAL;
    Workspace& ws = ctx->ws;
    hipStream_t s = ctx->stream;
    const size_t N = ctx->last_n;
    API_HIPCHK(hipSetDevice(ctx->device));
    if (ctx->last_mem == WFA_DEVICE) {
        int rc = ws.ensure(ws.out_offsets, (N + 1) * 8);
        if (rc == WFA_OK) rc = ws.ensure(ws.scan_tmp, scan_temp_bytes(N + 1) + 64);
        if (rc != WFA_OK) return rc;
        uint64_t* off = ws.out_offsets.as<uint64_t>();
        API_HIPCHK(launch_scan(SCAN_U32, ws.nruns.ptr, N, off, ws.scan_tmp.ptr, s));
        API_HIPCHK(launch_compact(ws.run_src.as<uint64_t>(),
                                  ws.slots.as<uint32_t>(), ws.slots2.as<uint32_t>(),
                                  ws.gen_runs.as<uint32_t>(), off, N, runs,
                                  capacity, nullptr, s));
        if (offsets)
            API_HIPCHK(hipMemcpyAsync(offsets, off, (N + 1) * 8, hipMemcpyDeviceToDevice, s));
    } else {
        // the host-memory pipeline keeps the whole batch's runs and offsets
        // on the device
        if (ctx->last_total)
            API_HIPCHK(hipMemcpyAsync(runs, ws.out_runs.ptr, ctx->last_total * 4,
                                      hipMemcpyDeviceToHost, s));
        if (offsets)
            API_HIPCHK(hipMemcpyAsync(offsets, ws.host_off.ptr, (N + 1) * 8, hipMemcpyDeviceToHost,
                                      s));
    }
    API_HIPCHK(hipStreamSynchronize(s));
    return WFA_OK;
}

extern "C" int wfa_host_alloc(size_t bytes, void** out) {
    if (!out) return WFA_E_INVAL;
    *out = nullptr;
    if (hipHostMalloc(out, bytes ? bytes : 1, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        return WFA_E_NOMEM;
    }
    return WFA_OK;
}

extern "C" void wfa_host_free(void* ptr) {
    if (ptr) (void)hipHostFree(ptr);
}

extern "C" int wfa_pack2bit(wfa_ctx* ctx, const uint8_t* ascii, const uint64_t* starts,
                            const uint32_t* lens, size_t count, uint64_t* words,
                            size_t words_capacity, uint64_t* word_starts, size_t* total_words,
                            int64_t* bad_index, void* stream) {
    if (bad_index) *bad_index = -1;
    if (total_words) *total_words = 0;
    if (!ctx || (count && (!ascii || !starts || !lens || !word_starts))) return WFA_E_INVAL;
    if (!count) return WFA_OK;
    Workspace& ws = ctx->ws;
    hipStream_t s = ctx->stream;
    API_HIPCHK(hipSetDevice(ctx->device));
    if (stream) {
        API_HIPCHK(hipEventRecord(ctx->ev[7], (hipStream_t)stream));
        API_HIPCHK(hipStreamWaitEvent(s, ctx->ev[7], 0));
    }
    int rc = ws.ensure(ws.scan_tmp, scan_temp_bytes(count + 1) + 64);
    if (rc == WFA_OK) rc = ws.ensure(ws.flags, sizeof(DevFlags));
    if (rc != WFA_OK) return rc;
    API_HIPCHK(launch_scan(SCAN_WORDS_LEN, lens, count, word_starts, ws.scan_tmp.ptr, s));
    uint64_t total = 0;
    API_HIPCHK(hipMemcpyAsync(&total, word_starts + count, 8, hipMemcpyDeviceToHost, s));
    API_HIPCHK(hipStreamSynchronize(s));
    if (total_words) *total_words = total;
    if (total > words_capacity || (total && !words)) return WFA_E_CAPACITY;
    DevFlags* fl = ws.flags.as<DevFlags>();
    API_HIPCHK(launch_fill_u64((uint64_t*)&fl->err_pair, ~0ull, 1, s));
    API_HIPCHK(launch_pack_seqs(ascii, starts, lens, count, word_starts, total, words,
                                &fl->err_pair, s));
    unsigned long long err = 0;
    API_HIPCHK(hipMemcpyAsync(&err, &fl->err_pair, 8, hipMemcpyDeviceToHost, s));
    if (stream) {
        API_HIPCHK(hipEventRecord(ctx->ev[6], s));
        API_HIPCHK(hipStreamWaitEvent((hipStream_t)stream, ctx->ev[6], 0));
    }
    API_HIPCHK(hipStreamSynchronize(s));
    if (err != ~0ull) {
        if (bad_index) *bad_index = (int64_t)err;
        return WFA_E_ALPHABET;
    }
    return WFA_OK;
}
