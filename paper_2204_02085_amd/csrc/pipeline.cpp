// Host-memory batches as a three-stage pipeline over chunks of consecutive
// pairs: copy in (stream h2d, a library thread), align (the engine's stream,
// the calling thread, the device-memory path once per chunk) and copy out
// (stream d2h, a second library thread).  While chunk k aligns, chunk k+1's
// inputs travel to the device and chunk k-1's results travel back.
//
// The device keeps a copy of the whole batch: descriptors and sequence bytes
// at the caller's own offsets (so the descriptors need no rewriting), the
// scores, the offsets counted from the batch's first run, and every run, so
// wfa_copy_last_cigars can serve a call that ran out of run capacity.
//
// Page-locked caller buffers move by DMA directly; pageable ones pass
// through two page-locked staging slots per direction that a pool of host
// threads fills or empties while the DMA engine works on the other slot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/wfa.h"
#include "copy_pool.h"
#include "internal.h"
#include "kernels.h"

using namespace wfa;

namespace {

#define HIPCHK(x)                                                                   \
    do {                                                                            \
        hipError_t _e = (x);                                                        \
        if (_e != hipSuccess) {                                                     \
            std::fprintf(stderr, "libwfa: %s failed (%s:%d): %s\n", #x, __FILE__,   \
                         __LINE__, hipGetErrorString(_e));                          \
            (void)hipGetLastError();                                                \
            return WFA_E_DEVICE;                                                    \
        }                                                                           \
    } while (0)

#define RCCHK(x)                     \
    do {                             \
        int _r = (x);                \
        if (_r != WFA_OK) return _r; \
    } while (0)

// Default chunk: a quarter of the batch within [MIN_CHUNK, MAX_CHUNK] pairs.
// Fewer, larger chunks amortise the per-chunk host round trips; more,
// smaller ones shorten the pipeline's fill and drain (on one MI355X over
// PCIe, 5 M pairs of 100 bp run fastest in 4 chunks).
constexpr size_t MIN_CHUNK = 262144;
constexpr size_t MAX_CHUNK = 2097152;
constexpr size_t MAX_CHUNKS = 1024;  // bounds the host-side bookkeeping

// Whether `p` is page-locked host memory the DMA engines can read directly.
bool page_locked(const void* p) {
    if (!p) return true;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeHost;
}

constexpr size_t STAGE_SLOT = (size_t)32 << 20;  // bytes per staging slot (two per direction)

double wall_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Chunk {
    size_t first = 0, n = 0;    // pairs [first, first + n)
    uint64_t p_lo = 0, p_hi = 0;  // pattern units first needed by this chunk
    uint64_t t_lo = 0, t_hi = 0;  // text units first needed by this chunk
    uint64_t run_base = 0;        // first run of the chunk in the batch
    uint64_t runs = 0;            // runs of the chunk
};

// Progress of the three stages; a stage waits for the one before it.
struct Progress {
    std::mutex mu;
    std::condition_variable cv;
    size_t in_issued = 0;  // chunks whose input copies are enqueued
    size_t aligned = 0;    // chunks whose results are on the device
    size_t out_done = 0;   // chunks whose results are in host memory
    int error = WFA_OK;    // first failure of any stage; stops the others

    // Wait until `*field >= v`; false once any stage has failed.
    bool wait(const size_t* field, size_t v) {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return error != WFA_OK || *field >= v; });
        return error == WFA_OK;
    }
    void publish(size_t* field, size_t v) {
        {
            std::lock_guard<std::mutex> lk(mu);
            *field = v;
        }
        cv.notify_all();
    }
    void fail(int rc) {
        {
            std::lock_guard<std::mutex> lk(mu);
            if (error == WFA_OK) error = rc;
        }
        cv.notify_all();
    }
    bool failed() {
        std::lock_guard<std::mutex> lk(mu);
        return error != WFA_OK;
    }
};

// End (in units of the encoding) of the pattern and text bytes each chunk's
// pairs reach, and the first pair whose length exceeds the limit.  Slices of
// the descriptor array are scanned by up to 8 threads.
void scan_chunk_ends(const wfa_pair* pairs, size_t n, size_t chunk, bool ascii,
                     std::vector<uint64_t>& end_p, std::vector<uint64_t>& end_t,
                     int64_t* too_long) {
    const size_t K = end_p.size();
    unsigned T = 1;
    if (n >= ((size_t)1 << 18)) T = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
    std::vector<std::vector<uint64_t>> lp(T), lt(T);
    std::vector<int64_t> bad(T, -1);
    auto work = [&](unsigned t) {
        const size_t a = n * t / T, b = n * (t + 1) / T;
        lp[t].assign(K, 0);
        lt[t].assign(K, 0);
        for (size_t i = a; i < b; i++) {
            const wfa_pair& q = pairs[i];
            if (q.p_len > WFA_MAX_LENGTH || q.t_len > WFA_MAX_LENGTH) {
                if (bad[t] < 0) bad[t] = (int64_t)i;
                continue;
            }
            const size_t k = i / chunk;
            const uint64_t ep = q.p_start + (ascii ? q.p_len : (q.p_len + 31ull) / 32);
            const uint64_t et = q.t_start + (ascii ? q.t_len : (q.t_len + 31ull) / 32);
            lp[t][k] = std::max(lp[t][k], ep);
            lt[t][k] = std::max(lt[t][k], et);
        }
    };
    std::vector<std::thread> th;
    try {
        for (unsigned t = 1; t < T; t++) th.emplace_back(work, t);
    } catch (...) {
        for (auto& x : th) x.join();
        th.clear();
        for (unsigned t = 1; t < T; t++) work(t);
    }
    work(0);
    for (auto& x : th) x.join();
    *too_long = -1;
    for (unsigned t = 0; t < T; t++) {
        if (bad[t] >= 0 && *too_long < 0) *too_long = bad[t];
        for (size_t k = 0; k < K; k++) {
            end_p[k] = std::max(end_p[k], lp[t][k]);
            end_t[k] = std::max(end_t[k], lt[t][k]);
        }
    }
}

}  // namespace

int engine_align(Engine* e, const BatchIO& io, hipStream_t user_stream, size_t* cigar_needed,
                 int64_t* bad_pair) {
    const int rc = io.mem == WFA_HOST
                       ? engine_align_host(e, io, user_stream, cigar_needed, bad_pair)
                       : engine_align_device(e, io, user_stream, cigar_needed, bad_pair);
    if (rc == WFA_E_NOMEM) {
        // the buffers a batch that did not fit left behind would count
        // against every later batch: start the next one from nothing
        graph_cache_clear(e);
        e->ws.release_all();
    }
    return rc;
}

int engine_align_host(Engine* e, const BatchIO& io, hipStream_t user_stream, size_t* cigar_needed,
                      int64_t* bad_pair) {
    const double t_start = wall_ms();
    if (bad_pair) *bad_pair = -1;
    if (cigar_needed) *cigar_needed = 0;
    Pen pen;
    RCCHK(make_pen(io.pen, &pen));
    if (io.enc != WFA_ASCII && io.enc != WFA_PACKED2) return WFA_E_INVAL;
    if (io.mode != WFA_SCORE && io.mode != WFA_CIGAR) return WFA_E_INVAL;
    const bool cigar = io.mode == WFA_CIGAR;
    const size_t N = io.n;
    if (N > 0 && (!io.patterns || !io.texts || !io.pairs || !io.scores)) return WFA_E_INVAL;
    if (cigar && !io.offsets) return WFA_E_INVAL;
    if (cigar && io.capacity && !io.runs) return WFA_E_INVAL;
    if (N >= ((size_t)1 << 32) - 1) return WFA_E_INVAL;
    if (hipSetDevice(e->device) != hipSuccess) return WFA_E_DEVICE;
    std::memset(&e->last, 0, sizeof(e->last));
    e->last_valid = false;
    if (N == 0) {
        if (cigar) io.offsets[0] = 0;
        return WFA_OK;
    }

    // ---- chunks and the sequence ranges each one brings -----------------------
    size_t chunk = e->opt.host_chunk_pairs > 0
                       ? (size_t)e->opt.host_chunk_pairs
                       : std::min(MAX_CHUNK, std::max(MIN_CHUNK, (N + 3) / 4));
    chunk = std::max(chunk, (N + MAX_CHUNKS - 1) / MAX_CHUNKS);
    chunk = std::min(chunk, N);
    const size_t K = (N + chunk - 1) / chunk;
    const bool ascii = io.enc == WFA_ASCII;
    const size_t unit = ascii ? 1 : 8;
    std::vector<uint64_t> end_p(K, 0), end_t(K, 0);
    int64_t too_long = -1;
    scan_chunk_ends(io.pairs, N, chunk, ascii, end_p, end_t, &too_long);
    if (too_long >= 0) {
        if (bad_pair) *bad_pair = too_long;
        return WFA_E_TOO_LONG;
    }
    // chunk k copies what no earlier chunk has copied: everything below the
    // running maximum of the ends is on the device once its copies are done
    std::vector<Chunk> ch(K);
    uint64_t hp = 0, ht = 0;
    for (size_t k = 0; k < K; k++) {
        Chunk& c = ch[k];
        c.first = k * chunk;
        c.n = std::min(chunk, N - c.first);
        c.p_lo = hp;
        c.t_lo = ht;
        hp = std::max(hp, end_p[k]);
        ht = std::max(ht, end_t[k]);
        c.p_hi = hp;
        c.t_hi = ht;
    }

    // ---- device copy of the batch ------------------------------------------------
    Workspace& ws = e->ws;
    RCCHK(ws.ensure(ws.in_pairs, N * sizeof(wfa_pair)));
    RCCHK(ws.ensure(ws.in_p, hp * unit + 8));
    RCCHK(ws.ensure(ws.in_t, ht * unit + 8));
    RCCHK(ws.ensure(ws.out_scores, N * 4));
    if (cigar) {
        RCCHK(ws.ensure(ws.host_off, (N + 1) * 8));
        RCCHK(ws.ensure(ws.host_loff, (chunk + 1) * 8));
    }
    std::vector<hipEvent_t> ev_in(K, nullptr), ev_al(K, nullptr);
    auto destroy_events = [&]() {
        for (auto& v : ev_in)
            if (v) (void)hipEventDestroy(v);
        for (auto& v : ev_al)
            if (v) (void)hipEventDestroy(v);
    };
    for (size_t k = 0; k < K; k++) {
        if (hipEventCreateWithFlags(&ev_in[k], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ev_al[k], hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            destroy_events();
            return WFA_E_DEVICE;
        }
    }
    if (user_stream) {
        HIPCHK(hipEventRecord(e->ev[7], user_stream));
        HIPCHK(hipStreamWaitEvent(e->h2d, e->ev[7], 0));
    }

    // Caller memory that is not page-locked moves through page-locked
    // staging: two slots per direction, filled (inputs) or emptied (results)
    // by a pool of host threads while the DMA engine works on the other slot.
    const bool locked_in = page_locked(io.pairs) && page_locked(io.patterns) &&
                           page_locked(io.texts);
    const bool locked_out = page_locked(io.scores) &&
                            (!cigar || (page_locked(io.offsets) && page_locked(io.runs)));
    unsigned char* stage_in = nullptr;
    unsigned char* stage_out = nullptr;
    hipEvent_t sev[4] = {};
    auto destroy_stage_events = [&]() {
        for (auto& v : sev)
            if (v) (void)hipEventDestroy(v);
    };
    if (!locked_in || !locked_out) {
        RCCHK(ws.ensure_pinned(4 * STAGE_SLOT));
        stage_in = (unsigned char*)ws.pinned;
        stage_out = stage_in + 2 * STAGE_SLOT;
        for (auto& v : sev) {
            if (hipEventCreateWithFlags(&v, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                destroy_stage_events();
                destroy_events();
                return WFA_E_DEVICE;
            }
        }
    }
    const unsigned hc = std::max(1u, std::thread::hardware_concurrency());
    std::unique_ptr<CopyPool> pool_in, pool_out;
    // helper threads only for batches large enough to repay starting them
    const uint64_t in_bytes = N * sizeof(wfa_pair) + (hp + ht) * unit;
    const bool big = in_bytes >= ((uint64_t)64 << 20);
    if (!locked_in) pool_in.reset(new CopyPool(big ? std::min(7u, std::max(1u, hc / 2)) - 1 : 0));
    if (!locked_out) pool_out.reset(new CopyPool(big ? std::min(3u, std::max(1u, hc / 4)) - 1 : 0));
    bool in_used[2] = {false, false};
    int in_next = 0;
    // host -> device, on h2d (returns once the caller's bytes are read or staged)
    auto to_device = [&](void* dst, const void* src, size_t bytes) -> int {
        if (locked_in) {
            HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, e->h2d));
            return WFA_OK;
        }
        for (size_t off = 0; off < bytes; off += STAGE_SLOT) {
            const size_t len = std::min(STAGE_SLOT, bytes - off);
            const int sl = in_next;
            in_next ^= 1;
            if (in_used[sl]) HIPCHK(hipEventSynchronize(sev[sl]));
            unsigned char* slot = stage_in + sl * STAGE_SLOT;
            pool_in->copy(slot, (const unsigned char*)src + off, len);
            HIPCHK(hipMemcpyAsync((unsigned char*)dst + off, slot, len, hipMemcpyHostToDevice,
                                  e->h2d));
            HIPCHK(hipEventRecord(sev[sl], e->h2d));
            in_used[sl] = true;
        }
        return WFA_OK;
    };
    // device -> host, on d2h, after what d2h already waits for (returns with
    // the bytes in caller memory when staged, else with the copy enqueued)
    auto to_host = [&](void* dst, const void* src, size_t bytes) -> int {
        if (locked_out) {
            HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, e->d2h));
            return WFA_OK;
        }
        // piece i + 1 moves into one slot while piece i leaves the other
        size_t prev_off = 0, prev_len = 0;
        int prev_sl = -1, sl = 0;
        for (size_t off = 0;; off += STAGE_SLOT) {
            const size_t len = off < bytes ? std::min(STAGE_SLOT, bytes - off) : 0;
            if (len) {
                HIPCHK(hipMemcpyAsync(stage_out + sl * STAGE_SLOT, (const unsigned char*)src + off,
                                      len, hipMemcpyDeviceToHost, e->d2h));
                HIPCHK(hipEventRecord(sev[2 + sl], e->d2h));
            }
            if (prev_sl >= 0) {
                HIPCHK(hipEventSynchronize(sev[2 + prev_sl]));
                pool_out->copy((unsigned char*)dst + prev_off, stage_out + prev_sl * STAGE_SLOT,
                               prev_len);
            }
            if (!len) break;
            prev_sl = sl;
            prev_off = off;
            prev_len = len;
            sl ^= 1;
        }
        return WFA_OK;
    };

    Progress pr;
    // stage 1: inputs of every chunk, in order, on h2d
    auto copy_in = [&]() -> int {
        if (hipSetDevice(e->device) != hipSuccess) return WFA_E_DEVICE;
        for (size_t k = 0; k < K; k++) {
            if (pr.failed()) return WFA_OK;
            const Chunk& c = ch[k];
            RCCHK(to_device(ws.in_pairs.as<wfa_pair>() + c.first, io.pairs + c.first,
                            c.n * sizeof(wfa_pair)));
            if (c.p_hi > c.p_lo)
                RCCHK(to_device(ws.in_p.as<uint8_t>() + c.p_lo * unit,
                                (const uint8_t*)io.patterns + c.p_lo * unit,
                                (c.p_hi - c.p_lo) * unit));
            if (c.t_hi > c.t_lo)
                RCCHK(to_device(ws.in_t.as<uint8_t>() + c.t_lo * unit,
                                (const uint8_t*)io.texts + c.t_lo * unit, (c.t_hi - c.t_lo) * unit));
            HIPCHK(hipEventRecord(ev_in[k], e->h2d));
            pr.publish(&pr.in_issued, k + 1);
        }
        return WFA_OK;
    };
    // stage 3: results of every chunk, in order, on d2h
    auto copy_out = [&]() -> int {
        if (hipSetDevice(e->device) != hipSuccess) return WFA_E_DEVICE;
        for (size_t k = 0; k < K; k++) {
            if (!pr.wait(&pr.aligned, k + 1)) return WFA_OK;
            const Chunk& c = ch[k];
            HIPCHK(hipStreamWaitEvent(e->d2h, ev_al[k], 0));
            RCCHK(to_host(io.scores + c.first, ws.out_scores.as<int32_t>() + c.first, c.n * 4));
            if (cigar) {
                RCCHK(to_host(io.offsets + c.first, ws.host_off.as<uint64_t>() + c.first,
                              (c.n + 1) * 8));
                if (c.runs && c.run_base + c.runs <= io.capacity)
                    RCCHK(to_host(io.runs + c.run_base, ws.out_runs.as<uint32_t>() + c.run_base,
                                  c.runs * 4));
            }
            HIPCHK(hipStreamSynchronize(e->d2h));
            pr.publish(&pr.out_done, k + 1);
        }
        return WFA_OK;
    };
    // stage 2 (this thread): each chunk through the device-memory path
    wfa_stats sum{};
    uint64_t base = 0;
    int64_t chunk_bad = -1;
    auto align_all = [&]() -> int {
        for (size_t k = 0; k < K; k++) {
            if (!pr.wait(&pr.in_issued, k + 1)) return WFA_OK;
            Chunk& c = ch[k];
            HIPCHK(hipStreamWaitEvent(e->stream, ev_in[k], 0));
            uint64_t room = 0;
            if (cigar) {
                // room for this chunk's runs at the rate seen so far (16 per
                // pair before any); when the buffer must move, it is sized for
                // the rest of the batch, once the earlier chunks' runs have
                // left it
                const double rate = k ? (double)base / (double)c.first : 16.0;
                const uint64_t want = (uint64_t)(rate * 1.25 * (double)c.n) + 1024;
                if (ws.out_runs.bytes / 4 < base + want) {
                    if (!pr.wait(&pr.out_done, k)) return WFA_OK;
                    const uint64_t rest = (uint64_t)(rate * 1.25 * (double)(N - c.first)) + 1024;
                    RCCHK(ws.grow_keep(ws.out_runs, (base + std::max(want, rest) + 1) * 4, base * 4,
                                       e->stream));
                }
                room = ws.out_runs.bytes / 4 - base;
            }
            BatchIO sub{ws.in_p.ptr,
                        ws.in_t.ptr,
                        ws.in_pairs.as<wfa_pair>() + c.first,
                        c.n,
                        io.enc,
                        WFA_DEVICE,
                        io.pen,
                        io.mode,
                        ws.out_scores.as<int32_t>() + c.first,
                        cigar ? ws.out_runs.as<uint32_t>() + base : nullptr,
                        room,
                        cigar ? ws.host_loff.as<uint64_t>() : nullptr};
            sub.no_graph = true;
            size_t needed = 0;
            int64_t bad = -1;
            int rc = engine_align_device(e, sub, nullptr, &needed, &bad);
            if (rc == WFA_E_CAPACITY) {
                // the chunk's runs are held by the engine; compact them once
                // the buffer has grown
                if (!pr.wait(&pr.out_done, k)) return WFA_OK;
                RCCHK(ws.grow_keep(ws.out_runs, (base + needed + 1) * 4, base * 4, e->stream));
                HIPCHK(launch_compact(ws.run_src.as<uint64_t>(),
                                      ws.slots.as<uint32_t>(), ws.slots2.as<uint32_t>(),
                                      ws.gen_runs.as<uint32_t>(), ws.host_loff.as<uint64_t>(), c.n,
                                      ws.out_runs.as<uint32_t>() + base, needed, nullptr,
                                      e->stream));
                rc = WFA_OK;
            }
            if (rc != WFA_OK) {
                if (bad >= 0) chunk_bad = (int64_t)c.first + bad;
                return rc;
            }
            c.run_base = base;
            c.runs = cigar ? needed : 0;
            if (cigar)
                HIPCHK(launch_add_u64(ws.host_loff.as<uint64_t>(), base, c.n + 1,
                                      ws.host_off.as<uint64_t>() + c.first, e->stream));
            HIPCHK(hipEventRecord(ev_al[k], e->stream));
            base += c.runs;
            const wfa_stats& L = e->last;
            sum.short_pairs += L.short_pairs;
            sum.general_pairs += L.general_pairs;
            sum.requeued += L.requeued;
            sum.window = std::max(sum.window, L.window);
            sum.lanes_per_pair = std::max(sum.lanes_per_pair, L.lanes_per_pair);
            sum.step_cap = std::max(sum.step_cap, L.step_cap);
            sum.schedule = L.schedule;
            sum.ms_pack += L.ms_pack;
            sum.ms_align += L.ms_align;
            sum.ms_general += L.ms_general;
            sum.ms_compact += L.ms_compact;
            pr.publish(&pr.aligned, k + 1);
        }
        return WFA_OK;
    };

    int rc_in = WFA_OK, rc_out = WFA_OK, rc_al = WFA_OK;
    std::thread t_in, t_out;
    bool threaded = K > 1;
    if (threaded) {
        try {
            t_in = std::thread([&] {
                rc_in = copy_in();
                if (rc_in != WFA_OK) pr.fail(rc_in);
            });
            t_out = std::thread([&] {
                rc_out = copy_out();
                if (rc_out != WFA_OK) pr.fail(rc_out);
            });
        } catch (...) {
            pr.fail(WFA_E_NOMEM);
        }
        rc_al = pr.failed() ? WFA_OK : align_all();
        if (rc_al != WFA_OK) pr.fail(rc_al);
        if (t_in.joinable()) t_in.join();
        if (t_out.joinable()) t_out.join();
    } else {
        rc_in = copy_in();
        if (rc_in != WFA_OK) pr.fail(rc_in);
        if (rc_in == WFA_OK) rc_al = align_all();
        if (rc_al != WFA_OK) pr.fail(rc_al);
        if (rc_in == WFA_OK && rc_al == WFA_OK) rc_out = copy_out();
    }
    // nothing may still read or write caller memory after the call returns
    const bool synced = hipStreamSynchronize(e->h2d) == hipSuccess &&
                        hipStreamSynchronize(e->stream) == hipSuccess &&
                        hipStreamSynchronize(e->d2h) == hipSuccess;
    if (!synced) (void)hipGetLastError();
    destroy_events();
    destroy_stage_events();
    for (int rc : {rc_al, rc_in, rc_out}) {
        if (rc != WFA_OK) {
            if (bad_pair && chunk_bad >= 0) *bad_pair = chunk_bad;
            e->last_valid = false;
            return rc;
        }
    }
    if (!synced) return WFA_E_DEVICE;

    wfa_stats& L = e->last;
    L = sum;
    L.pairs = N;
    L.cigar_runs = base;
    L.host_chunks = (int32_t)K;
    L.graph_replayed = 0;
    L.ms_total = wall_ms() - t_start;
    e->last_valid = cigar;
    e->last_n = N;
    e->last_mem = WFA_HOST;
    e->last_total = base;
    if (cigar_needed) *cigar_needed = (size_t)base;
    if (cigar && base > io.capacity) return WFA_E_CAPACITY;
    return WFA_OK;
}
