// One batch in device memory: plan, pack, short-pair kernel (plain or
// persistent, with optional bucketing and graph replay), general kernel for
// whatever the short kernel hands over, CIGAR offsets and compaction.  Host
// memory batches go through the chunk pipeline, which calls this per chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/wfa.h"
#include "internal.h"
#include "kernels.h"

using namespace wfa;

namespace {

constexpr uint32_t SHORT_MAX_LEN = 2400;  // longest sequence the short kernel stages in LDS

#define HIPCHK(x)                                                  \
    do {                                                           \
        hipError_t _e = (x);                                       \
        if (_e != hipSuccess) {                                    \
            report_hip_error(_e, #x, __FILE__, __LINE__);          \
            (void)hipGetLastError();                               \
            return WFA_E_DEVICE;                                   \
        }                                                          \
    } while (0)

void report_hip_error(hipError_t e, const char* what, const char* file, int line) {
    std::fprintf(stderr, "libwfa: %s failed (%s:%d): %s\n", what, file, line,
                 hipGetErrorString(e));
}

#define RCCHK(x)                  \
    do {                          \
        int _r = (x);             \
        if (_r != WFA_OK) return _r; \
    } while (0)

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

double ev_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();
        return 0.0;
    }
    return ms;
}

int auto_window(uint32_t max_len) {
    if (max_len <= 160) return 32;
    if (max_len <= 400) return 64;
    if (max_len <= 1200) return 128;
    if (max_len <= SHORT_MAX_LEN) return 256;
    return 0;
}

template <class F>
int capture_graph(hipStream_t s, F&& body, hipGraph_t* graph, hipGraphExec_t* exec) {
    *graph = nullptr;
    *exec = nullptr;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const int rc = body(s);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(s, &g);
    if (rc != WFA_OK || ce != hipSuccess || !g) {
        if (ce != hipSuccess) report_hip_error(ce, "hipStreamEndCapture", __FILE__, __LINE__);
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        return rc != WFA_OK ? rc : WFA_E_DEVICE;
    }
    const hipError_t ie = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        report_hip_error(ie, "hipGraphInstantiate", __FILE__, __LINE__);
        (void)hipGetLastError();
        (void)hipGraphDestroy(g);
        *exec = nullptr;
        return WFA_E_DEVICE;
    }
    *graph = g;
    return WFA_OK;
}

struct Dev {
    const PairDesc* pairs;    // descriptors of the packed words
    const uint64_t* pw;
    const uint64_t* tw;
    int32_t* scores;
    uint32_t* runs;
    uint64_t* offsets;
    uint64_t capacity;
};

// Pairs in `pending` on the workgroup-per-pair kernel, chunked by the budget;
// pairs whose slice is too small are retried with a 4x slice.
// A pair the kernel gives up on ends the call with WFA_E_LIMIT and its index
// in *gave_up_pair.
int run_general(Engine* e, const Pen& pen, bool cigar, const Dev& d, const BatchStats& st,
                std::vector<uint32_t> pending, uint64_t& gen_used, hipStream_t s,
                uint64_t* general_done, uint64_t* requeued, int64_t* gave_up_pair) {
    (void)st;
    Workspace& ws = e->ws;
    const uint64_t R = (uint64_t)pen.pre + 1;
    RCCHK(ws.ensure(ws.flags, sizeof(DevFlags)));
    DevFlags* flags = ws.flags.as<DevFlags>();

    // lengths of the pending pairs (the descriptors live on the device)
    std::vector<uint32_t> plen(pending.size()), tlen(pending.size());
    {
        RCCHK(ws.ensure(ws.jobs, pending.size() * 4));
        RCCHK(ws.ensure(ws.gen_tmp, pending.size() * 8));
        HIPCHK(hipMemcpyAsync(ws.jobs.ptr, pending.data(), pending.size() * 4,
                              hipMemcpyHostToDevice, s));
        HIPCHK(launch_pair_lengths(d.pairs, ws.jobs.as<uint32_t>(), pending.size(),
                                   ws.gen_tmp.as<uint32_t>(), s));
        std::vector<uint32_t> lens(2 * pending.size());
        HIPCHK(hipMemcpyAsync(lens.data(), ws.gen_tmp.ptr, lens.size() * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (size_t i = 0; i < pending.size(); i++) {
            plen[i] = lens[2 * i];
            tlen[i] = lens[2 * i + 1];
        }
    }
    // Longest pairs first: a launch then holds pairs of similar size, its
    // slices are sized for its own longest pair (short pairs run many at a
    // time), and the long pairs start early.
    struct Job {
        uint32_t pair, n, m;
    };
    std::vector<Job> jobs(pending.size());
    for (size_t i = 0; i < pending.size(); i++) jobs[i] = {pending[i], plen[i], tlen[i]};
    std::stable_sort(jobs.begin(), jobs.end(), [](const Job& a, const Job& b) {
        return (uint64_t)a.n + a.m > (uint64_t)b.n + b.m;
    });
    // CIGAR history, first guess: a pair at 10 % divergence (score about
    // 0.1 * L times the mean edit cost) keeps ~s'^2 / e' cells of 4.5 bytes
    // (offset and record; 2.5 with 16-bit offsets) plus a 16-byte step-table
    // entry per step, and its runs
    // Checkpoint mode (CIGAR): rows of R steps every ck steps, each of at most
    // 2s + 1 diagonals at step s, so ~3 R rb sg^2 / ck bytes of checkpoints;
    // a segment buffer of (ck + R) rows of 2 (ck + R - 1) / e + 1 columns
    // (M, I, D and a record byte each); the step table and the runs.
    // By default (general_checkpoint 0) a launch keeps the full history when
    // the arena holds that for every pair left, else checkpoints every 128
    // steps.
    auto ck_for = [&](bool memory_bound) -> int {
        if (!cigar) return 0;
        int c = e->opt.general_checkpoint;
        if (c < 0) return 0;
        if (c == 0) c = memory_bound ? 128 : 0;
        if (c == 0) return 0;
        c = std::max<int>(c, (int)R);  // checkpoint windows never overlap
        if (c + (int)R > GENERAL_SEG_ROWS || c > GENERAL_CKPT_MAX) return 0;
        return c;
    };
    auto seg_bytes_for = [&](int ck, uint64_t rb) -> double {
        if (!ck) return 0.0;
        const uint64_t wc = 2 * ((ck + R - 1) / (uint64_t)pen.e) + 1;
        return (double)((ck + R) * ((wc * (3 * rb + 1) + 15) & ~(uint64_t)15));
    };
    auto hist_est = [&](uint32_t n, uint32_t m, int ck, uint64_t rb) -> double {
        const double L = std::max(n, m);
        const double sg = 0.14 * L * (pen.x + 2.0 * pen.oe) / 3.0 + pen.oe;
        if (ck)
            return 3.0 * (double)R * (double)rb * sg * sg / ck + 64.0 * R * sg / ck +
                   seg_bytes_for(ck, rb) + 16.0 * sg + 4.0 * ((double)n + m + 1) + 4096.0;
        const double cellb = m < 0xFFFF ? 2.5 : 4.5;
        return cellb * sg * sg / pen.e + 32.0 * sg + 4.0 * ((double)n + m + 1) + 4096.0;
    };
    // After each launch the guess is scaled by 1.25x the largest ratio of
    // used to guessed bytes seen so far (never above the guess itself; one
    // scale per mode), so batches less divergent than the guess run more
    // pairs at a time; pairs whose slice is still too small are re-run with 4x
    double scale_seen[2] = {0.0, 0.0}, hist_scale[2] = {1.0, 1.0};
    auto slice_for = [&](uint32_t n, uint32_t m, uint64_t mult, uint64_t rb, int ck) -> uint64_t {
        const uint64_t nm1 = (uint64_t)n + m + 1;
        uint64_t sl;
        sl = (R + 1) * ((3 * rb * (nm1 + 2) + 15) & ~(uint64_t)15);  // ring slots, a NULL slot
        if (cigar && e->opt.general_slice_kib > 0)  // the caller's first guess
            sl += (uint64_t)e->opt.general_slice_kib * 1024 * mult + (uint64_t)seg_bytes_for(ck, rb);
        else if (cigar)
            sl += (uint64_t)std::min(std::max(hist_est(n, m, ck, rb) * hist_scale[ck ? 1 : 0],
                                              16.0 * 1024 + seg_bytes_for(ck, rb)),
                                     64.0 * 1024 * 1024 + seg_bytes_for(ck, rb)) * mult;
        return (sl + 255) & ~(uint64_t)255;
    };

    // The arena keeps whatever size it reached (re-allocating tens of GB per
    // batch costs more than the alignment); it grows only when the current
    // slices do not fit, and never past 3/4 of the budget left by the other
    // buffers, so staging and run buffers of later batches still fit.
    uint64_t mult = 1;
    int attempts = 0;
    size_t launches = 0, min_conc = ~(size_t)0;
    const size_t n_pending = jobs.size();
    HIPCHK(launch_fill_u64((uint64_t*)&flags->gave_up, ~0ull, 1, s));
    while (!jobs.empty()) {
        // 16-bit ring rows for a launch whose texts are all shorter than
        // 32767 bases: the largest text length from each position on
        std::vector<uint32_t> suffix_m(jobs.size() + 1, 0);
        for (size_t i = jobs.size(); i-- > 0;) suffix_m[i] = std::max(suffix_m[i + 1], jobs[i].m);
        if (++attempts > 40) {
            std::fprintf(stderr, "libwfa: %zu pairs still failing after 40 attempts\n", jobs.size());
            return WFA_E_NOMEM;
        }
        std::vector<Job> failed;
        for (size_t off = 0; off < jobs.size();) {
            const Job& head = jobs[off];  // the longest pair left
            const bool rows16 = suffix_m[off] < 32767;
            const uint64_t rb = rows16 ? 2 : 4;
            const size_t others = ws.total - ws.arena.bytes;
            const size_t arena_cap = ws.budget > others ? (ws.budget - others) / 4 * 3 : 0;
            // every pair gets a slice of its own size; full histories when the
            // arena holds them for every pair left (one launch), else
            // checkpoints: they let the pairs run in one launch, whose tail is
            // shorter than several launches' tails (100 k pairs of 1-10 kbp:
            // 580 ms in one launch against 611 ms in six)
            const size_t left = std::min(jobs.size() - off, (size_t)1 << 20);
            double full_bytes = 0;
            for (size_t i = 0; i < left; i++)
                full_bytes += (double)slice_for(jobs[off + i].n, jobs[off + i].m, mult, rb, 0);
            const bool memory_bound = full_bytes > (double)std::max(arena_cap, ws.arena.bytes);
            const int ck = ck_for(memory_bound);
            std::vector<uint64_t> soff(left + 1, 0);
            for (size_t i = 0; i < left; i++)
                soff[i + 1] = soff[i] + slice_for(jobs[off + i].n, jobs[off + i].m, mult, rb, ck);
            const uint64_t head_slice = soff[1];
            const size_t want = soff[left];
            if (ws.arena.bytes < want && ws.arena.bytes < arena_cap) {
                const size_t target = std::min(want, arena_cap);
                if (target > ws.arena.bytes && target >= head_slice) {
                    ws.release(ws.arena);
                    // the device may hold less than the budget: halve until it fits
                    size_t t = target;
                    int rc = ws.ensure(ws.arena, t);
                    while (rc != WFA_OK && t / 2 >= head_slice) {
                        t /= 2;
                        rc = ws.ensure(ws.arena, t);
                    }
                    RCCHK(rc);
                }
            }
            // the pairs whose slices fit in the arena, in order
            size_t conc = (size_t)(std::upper_bound(soff.begin(), soff.end(), (uint64_t)ws.arena.bytes) -
                                   soff.begin()) - 1;
            if (e->opt.general_pairs > 0) conc = std::min(conc, (size_t)e->opt.general_pairs);
            conc = std::min(conc, left);
            if (conc == 0) {
                std::fprintf(stderr, "libwfa: general kernel slice %zu B exceeds the arena (%zu B, "
                                     "budget %zu B)\n", (size_t)head_slice, ws.arena.bytes, ws.budget);
                return WFA_E_NOMEM;
            }
            const size_t nj = conc;
            launches++;
            min_conc = std::min(min_conc, conc);
            const uint32_t max_len = std::max(head.n, head.m);
            const uint32_t lds_words = (head.n + 31) / 32 + 1 + (head.m + 31) / 32 + 1;
            const bool seq_lds = (uint64_t)lds_words * 8 <= 48 * 1024;
            const int lds_bytes = seq_lds ? (int)(lds_words * 8) : 0;
            // Threads per pair above 600 bases, by the pairs in the launch: a
            // step's chain of ring reads, cells and barrier is latency-bound,
            // so a launch with many pairs runs faster with more pairs per CU
            // (100 k pairs of 1-10 kbp: 446 ms with 256 threads against 568 ms
            // with 512 and 1136 ms with 1024), while one with few pairs ends
            // when its longest pair does, sooner with more threads on it (1-10
            // kbp: 256 pairs 12.1 ms with 1024 threads against 24.2 ms with
            // 256; 4096 pairs 23.5 ms with 512 against 32.4 ms; 8192 pairs
            // 36.4 ms with 256 against 44.6 ms with 512)
            const size_t per_cu = (nj + e->num_cus - 1) / e->num_cus;
            const int bt = max_len <= 600 ? 64 : per_cu <= 8 ? 1024 : per_cu <= 24 ? 512 : 256;

            std::vector<uint32_t> ids(nj);
            for (size_t i = 0; i < nj; i++) ids[i] = jobs[off + i].pair;
            RCCHK(ws.ensure(ws.jobs, nj * 4));
            RCCHK(ws.ensure(ws.job_nruns, nj * 4));
            RCCHK(ws.ensure(ws.job_offsets, (nj + 1) * 8));
            RCCHK(ws.ensure(ws.fail_list, nj * 4));
            if (cigar) {
                RCCHK(ws.ensure(ws.gen_state, nj * sizeof(GenJobState)));
                RCCHK(ws.ensure(ws.job_used, nj * 8));
                HIPCHK(launch_fill_u64(ws.job_used.as<uint64_t>(), 0ull, nj, s));
            }
            RCCHK(ws.ensure(ws.scan_tmp, scan_temp_bytes(nj) + 64));
            RCCHK(ws.ensure(ws.gen_slices, (nj + 1) * 8));
            HIPCHK(hipMemcpyAsync(ws.jobs.ptr, ids.data(), nj * 4, hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(ws.gen_slices.ptr, soff.data(), (nj + 1) * 8, hipMemcpyHostToDevice,
                                  s));
            HIPCHK(launch_fill_u32(ws.job_nruns.as<uint32_t>(), 0u, nj, s));
            HIPCHK(launch_fill_u32(&flags->fail_count, 0u, 1, s));
            GeneralArgs g{};
            g.pairs = d.pairs;
            g.pw = d.pw;
            g.tw = d.tw;
            g.jobs = ws.jobs.as<uint32_t>();
            g.num_jobs = (uint32_t)nj;
            g.pen = pen;
            g.ends = e->ends;
            g.cigar = cigar ? 1 : 0;
            g.arena = ws.arena.as<uint8_t>();
            g.slice_off = ws.gen_slices.as<uint64_t>();
            g.scores = d.scores;
            g.nruns = ws.nruns.as<uint32_t>();
            g.run_src = ws.run_src.as<uint64_t>();
            g.job_nruns = ws.job_nruns.as<uint32_t>();
            g.job_used = cigar ? ws.job_used.as<uint64_t>() : nullptr;
            g.fail_list = ws.fail_list.as<uint32_t>();
            g.fail_count = &flags->fail_count;
            g.gave_up = &flags->gave_up;
            g.step_limit = e->opt.general_step_limit;
            g.ckpt = ck;
            g.jstate = cigar ? ws.gen_state.as<GenJobState>() : nullptr;
            g.heur = e->heur;
            HIPCHK(launch_general(g, bt, seq_lds, lds_bytes, rows16, s));
            uint32_t nfail = 0;
            unsigned long long gave_up = ~0ull;
            HIPCHK(hipMemcpyAsync(&nfail, &flags->fail_count, 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(&gave_up, &flags->gave_up, 8, hipMemcpyDeviceToHost, s));
            std::vector<uint64_t> used(cigar ? nj : 0);
            if (cigar)
                HIPCHK(hipMemcpyAsync(used.data(), ws.job_used.ptr, nj * 8, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            // the flag is never reset within the call: after the last launch
            // it holds the lowest pair index any launch gave up on
            if (gave_up != ~0ull) *gave_up_pair = (int64_t)gave_up;
            if (cigar) {
                const int mi = ck ? 1 : 0;
                for (size_t i = 0; i < nj; i++)
                    if (used[i])
                        scale_seen[mi] = std::max(
                            scale_seen[mi], (double)used[i] / hist_est(jobs[off + i].n, jobs[off + i].m,
                                                                        ck, rows16 ? 2 : 4));
                if (scale_seen[mi] > 0)
                    hist_scale[mi] = std::min(1.0, std::max(1.0 / 16, 1.25 * scale_seen[mi]));
            }
            if (nfail) {
                std::vector<uint32_t> f(nfail);
                HIPCHK(hipMemcpy(f.data(), ws.fail_list.ptr, nfail * 4ull, hipMemcpyDeviceToHost));
                std::sort(f.begin(), f.end());
                for (size_t i = 0; i < nj; i++)
                    if (std::binary_search(f.begin(), f.end(), jobs[off + i].pair))
                        failed.push_back(jobs[off + i]);
            }
            *general_done += nj - nfail;
            if (cigar) {
                // gather this chunk's runs out of the arena before it is reused
                HIPCHK(launch_scan(SCAN_U32, ws.job_nruns.ptr, nj, ws.job_offsets.as<uint64_t>(),
                                   ws.scan_tmp.ptr, s));
                uint64_t chunk_runs = 0;
                HIPCHK(hipMemcpyAsync(&chunk_runs, ws.job_offsets.as<uint64_t>() + nj, 8,
                                      hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                RCCHK(ws.grow_keep(ws.gen_runs, (gen_used + chunk_runs + 1) * 4, gen_used * 4, s));
                HIPCHK(launch_gather_general(ws.jobs.as<uint32_t>(), nj, ws.job_nruns.as<uint32_t>(),
                                             ws.run_src.as<uint64_t>(), ws.arena.as<uint8_t>(), 0,
                                             ws.job_offsets.as<uint64_t>(), gen_used,
                                             ws.gen_runs.as<uint32_t>(), s));
                gen_used += chunk_runs;
            }
            off += nj;
        }
        *requeued += failed.size();
        jobs.swap(failed);
        mult *= 4;
    }
    if (*gave_up_pair >= 0) return WFA_E_LIMIT;
    if (std::getenv("WFA_DEBUG"))
        std::fprintf(stderr,
                     "libwfa general: %zu pairs, %zu launches (fewest pairs in one: %zu), "
                     "%d rounds, arena %.2f GiB, history scale %.3f (checkpoints %.3f)\n",
                     n_pending, launches, min_conc, attempts, ws.arena.bytes / 1073741824.0,
                     hist_scale[0], hist_scale[1]);
    return WFA_OK;
}

}  // namespace

bool GraphKey::operator==(const GraphKey& o) const {
    for (int i = 0; i < 8; i++)
        if (p[i] != o.p[i]) return false;
    for (int i = 0; i < 18; i++)
        if (ints[i] != o.ints[i]) return false;
    return n == o.n && capacity == o.capacity && form == o.form;
}

void destroy_graph(GraphEntry& g) {
    if (g.exec_all) (void)hipGraphExecDestroy(g.exec_all);
    if (g.graph_all) (void)hipGraphDestroy(g.graph_all);
    if (g.exec_pre) (void)hipGraphExecDestroy(g.exec_pre);
    if (g.graph_pre) (void)hipGraphDestroy(g.graph_pre);
    if (g.exec_post) (void)hipGraphExecDestroy(g.exec_post);
    if (g.graph_post) (void)hipGraphDestroy(g.graph_post);
    g = GraphEntry{};
}

void graph_cache_clear(Engine* e) {
    for (auto& g : e->graphs) destroy_graph(g);
    e->graphs.clear();
}

int engine_align_device(Engine* e, const BatchIO& io, hipStream_t user_stream,
                        size_t* cigar_needed, int64_t* bad_pair) {
    const double t_start = now_ms();
    if (bad_pair) *bad_pair = -1;
    if (cigar_needed) *cigar_needed = 0;
    Pen pen;
    RCCHK(make_pen(io.pen, &pen));
    if (io.enc != WFA_ASCII && io.enc != WFA_PACKED2) return WFA_E_INVAL;
    if (io.mem != WFA_DEVICE) return WFA_E_INVAL;
    if (io.mode != WFA_SCORE && io.mode != WFA_CIGAR) return WFA_E_INVAL;
    const bool cigar = io.mode == WFA_CIGAR;
    const size_t N = io.n;
    if (N > 0 && (!io.patterns || !io.texts || !io.pairs || !io.scores)) return WFA_E_INVAL;
    if (cigar && !io.offsets) return WFA_E_INVAL;
    if (cigar && io.capacity && !io.runs) return WFA_E_INVAL;
    if (N >= ((size_t)1 << 32) - 1) return WFA_E_INVAL;
    if (hipSetDevice(e->device) != hipSuccess) return WFA_E_DEVICE;
    Workspace& ws = e->ws;
    hipStream_t s = e->stream;
    std::memset(&e->last, 0, sizeof(e->last));
    e->last_valid = false;
    if (user_stream) {
        HIPCHK(hipEventRecord(e->ev[7], user_stream));
        HIPCHK(hipStreamWaitEvent(s, e->ev[7], 0));
    }
    // `idle`: nothing was enqueued on the engine's stream since its last
    // synchronisation, so the host need not wait again
    auto finish_user = [&](bool idle = false) -> int {
        if (user_stream) {
            HIPCHK(hipEventRecord(e->ev[6], s));
            HIPCHK(hipStreamWaitEvent(user_stream, e->ev[6], 0));
        }
        if (!idle) HIPCHK(hipStreamSynchronize(s));
        return WFA_OK;
    };

    if (N == 0) {
        if (cigar) HIPCHK(launch_fill_u64(io.offsets, 0ull, 1, s));
        return finish_user();
    }

    const PairDesc* in_pairs = (const PairDesc*)io.pairs;
    const void* in_p = io.patterns;
    const void* in_t = io.texts;
    Dev d{};
    d.scores = io.scores;
    d.offsets = io.offsets;
    d.runs = io.runs;
    d.capacity = io.capacity;

    // ---- batch facts -------------------------------------------------------
    RCCHK(ws.ensure(ws.stats, sizeof(BatchStats) * (1 + STATS_BLOCKS)));
    RCCHK(ws.ensure(ws.flags, sizeof(DevFlags)));
    static_assert(sizeof(BatchStats) <= 128 && sizeof(DevFlags) <= 128, "read-back slots");
    unsigned char* rb = (unsigned char*)e->readback + 128;  // the flags (with the run total)
    // Speculative start: the previous call's whole-pass graph, if this call
    // matches everything that graph was planned under except the batch facts
    // (packed input, so no packing depends on them); kept below only if the
    // facts lead to the same plan, else the call runs as planned and
    // overwrites every output.
    const GraphEntry* spec_ent = nullptr;
    if (e->spec.valid && !io.no_graph && io.enc == WFA_PACKED2) {
        const GraphKey& k = e->spec.key;
        const void* ptrs[7] = {in_pairs, in_p, in_t, io.scores, io.runs, io.offsets,
                               (const void*)(uintptr_t)ws.generation};
        bool same = k.n == N && k.capacity == (uint64_t)io.capacity && k.form == 1 &&
                    k.ints[0] == (int)io.enc && k.ints[1] == (int)io.mode && k.ints[2] == pen.x &&
                    k.ints[3] == pen.oe && k.ints[4] == pen.e && k.ints[5] == pen.g &&
                    std::memcmp(&e->spec.opt, &e->opt, sizeof(wfa_options)) == 0 &&
                    std::memcmp(&e->spec.ends, &e->ends, sizeof(e->ends)) == 0 &&
                    std::memcmp(&e->spec.heur, &e->heur, sizeof(e->heur)) == 0;
        for (int i = 0; i < 7 && same; i++) same = k.p[i] == ptrs[i];
        if (same)
            for (auto& g : e->graphs)
                if (g.key == k && g.exec_all) spec_ent = &g;
    }
    GraphKey spec_key;
    BatchStats st;
    // with a speculative launch the batch facts run on the copy stream,
    // beside the graph (both only read the inputs); the graph is submitted
    // first, so the device starts it before the host queues the facts
    hipStream_t sf = spec_ent ? e->h2d : s;
    if (spec_ent) {
        HIPCHK(hipEventRecord(e->ev[9], s));  // after any wait on the caller's stream
        spec_key = spec_ent->key;
        HIPCHK(hipEventRecord(e->ev[0], s));
        HIPCHK(hipGraphLaunch(spec_ent->exec_all, s));
        HIPCHK(hipEventRecord(e->ev[1], s));
        HIPCHK(hipMemcpyAsync(rb, ws.flags.ptr, sizeof(DevFlags), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamWaitEvent(sf, e->ev[9], 0));
    }
    HIPCHK(launch_batch_stats(in_pairs, N, ws.stats.as<BatchStats>(), WFA_MAX_LENGTH, sf));
    HIPCHK(hipMemcpyAsync(e->readback, ws.stats.ptr, sizeof(st), hipMemcpyDeviceToHost, sf));
    if (spec_ent) HIPCHK(hipStreamSynchronize(sf));
    e->spec.valid = false;  // set again once this call has planned and launched
    HIPCHK(hipStreamSynchronize(s));
    std::memcpy(&st, e->readback, sizeof(st));
    const double t_stats = now_ms();
    if (st.too_long) {
        if (bad_pair) *bad_pair = (int64_t)st.first_too_long;
        return WFA_E_TOO_LONG;
    }
    const uint32_t max_len = std::max(st.max_p, st.max_t);

    // ---- plan ------------------------------------------------------------
    int schedule = e->opt.schedule ? e->opt.schedule : WFA_SCHED_AUTO;
    int window = e->opt.window ? e->opt.window : auto_window(max_len);
    const bool global = e->ends.pb == 0 && e->ends.pe == 0 && e->ends.tb == 0 && e->ends.te == 0;
    if (!global && !e->opt.window && window) {
        // ends-free: the window must hold the free start diagonals -pb .. tb
        // with room to spare (it is centred between 0 and m - n)
        const uint32_t reach = std::max(std::min<uint32_t>((uint32_t)e->ends.pb, st.max_p),
                                        std::min<uint32_t>((uint32_t)e->ends.tb, st.max_t));
        while (window < 256 && (uint32_t)window < 2 * reach + 16) window *= 2;
        if ((uint32_t)window < 2 * reach + 16) window = 0;
    }
    ShortPlan sp;
    // the WF-adaptive heuristic runs on the general kernel alone (the
    // short-pair kernels are exact)
    bool use_short = schedule != WFA_SCHED_GENERAL && window != 0 && max_len <= SHORT_MAX_LEN &&
                     e->heur.mwl == 0;
    int lanes = 0;
    if (use_short) {
        const int cap = e->opt.step_cap ? e->opt.step_cap : default_cap(pen, window);
        lanes = e->opt.lanes_per_pair ? e->opt.lanes_per_pair : default_lanes(window);
        if (!short_shape_supported(window, lanes)) lanes = default_lanes(window);
        if (short_plan(e, pen, cigar, window, lanes, cap, max_len, &sp) != WFA_OK) use_short = false;
    }
    // The one-lane-per-pair kernel takes the first pass when it is built for
    // the penalties, the batch's lengths and the step cap (8 if the caller
    // asks for at most 8 steps, else 16), alignment is global, and no
    // short-kernel shape was asked for.  Pairs it cannot hold go to the
    // cascade from window 64 on, as from a 32-wide first pass.
    bool lane = false;
    if (use_short && global && e->opt.lane_kernel >= 0 && !e->opt.window && !e->opt.lanes_per_pair &&
        e->opt.step_cap <= 16) {
        const int lcap = (e->opt.step_cap > 0 && e->opt.step_cap <= 8) ? 8 : 16;
        // a workgroup's LDS (both sequences and, with CIGAR, the history of
        // every lane of its wavefronts) stays within 64 KiB
        int lbt = e->opt.block_threads ? e->opt.block_threads : 256;
        while (lbt > 64 && lane_lds_bytes(pen, lcap, cigar, lbt) > 64 * 1024) lbt -= 64;
        if (lane_supported(pen, lcap, max_len) && lane_lds_bytes(pen, lcap, cigar, lbt) <= 64 * 1024) {
            lane = true;
            window = 32;
            lanes = 1;
            sp = ShortPlan{};
            sp.window = 0;
            sp.lanes = 1;
            sp.cap = lcap;
            sp.slot_cap = 2 * (lcap / std::min(pen.x, pen.e) + 1) + 2;
            sp.block_threads = lbt;
            sp.lds_per_block = lane_lds_bytes(pen, lcap, cigar, lbt);
        }
    }
    const bool persistent = use_short && schedule != WFA_SCHED_PLAIN;
    const bool bucket = persistent && e->opt.bucket >= 0;
    // graphs: by default for the persistent schedule; the plain one only on request
    const bool graph = use_short && !io.no_graph && e->opt.use_graph >= 0 &&
                       (e->opt.use_graph > 0 || schedule == WFA_SCHED_AUTO ||
                        schedule == WFA_SCHED_PERSISTENT);

    // ---- buffers -----------------------------------------------------------
    const bool ascii = io.enc == WFA_ASCII;
    // ASCII sides whose sequences all need about the same number of words are
    // packed at a fixed stride (no word-start scan); others by scan
    const uint64_t mw_p = std::max<uint64_t>((st.max_p + 31) / 32, 1);
    const uint64_t mw_t = std::max<uint64_t>((st.max_t + 31) / 32, 1);
    const bool stride_p = ascii && N * mw_p <= st.words_p + st.words_p / 4 + 64;
    const bool stride_t = ascii && N * mw_t <= st.words_t + st.words_t / 4 + 64;
    if (ascii) {
        RCCHK(ws.ensure(ws.ws_p, (N + 1) * 8));
        RCCHK(ws.ensure(ws.ws_t, (N + 1) * 8));
        RCCHK(ws.ensure(ws.words_p, (stride_p ? N * mw_p : st.words_p) * 8 + 8));
        RCCHK(ws.ensure(ws.words_t, (stride_t ? N * mw_t : st.words_t) * 8 + 8));
        RCCHK(ws.ensure(ws.packed_pairs, N * sizeof(PairDesc)));
        d.pairs = ws.packed_pairs.as<PairDesc>();
        d.pw = ws.words_p.as<uint64_t>();
        d.tw = ws.words_t.as<uint64_t>();
    } else {
        d.pairs = in_pairs;
        d.pw = (const uint64_t*)in_p;
        d.tw = (const uint64_t*)in_t;
    }
    RCCHK(ws.ensure(ws.scan_tmp, scan_temp_bytes(N + 1) + 64));
    RCCHK(ws.ensure(ws.nruns, N * 4));
    RCCHK(ws.ensure(ws.run_src, N * 8));
    RCCHK(ws.ensure(ws.ovf_list, N * 4));
    if (use_short && cigar) RCCHK(ws.ensure(ws.slots, (size_t)N * sp.slot_cap * 4));
    if (bucket) {
        RCCHK(ws.ensure(ws.order, N * 4));
        RCCHK(ws.ensure(ws.keys, N * 4));
        RCCHK(ws.ensure(ws.hist, BUCKET_KEYS * 8));
    }
    // the bucket histogram, then the pairs of each key placed so far
    uint32_t* hist = bucket ? ws.hist.as<uint32_t>() : nullptr;
    uint32_t* taken = bucket ? hist + BUCKET_KEYS : nullptr;
    DevFlags* flags = ws.flags.as<DevFlags>();

    int grid = 1;
    int queue_chunk = 1;
    if (use_short) {
        // pairs per workgroup: lane groups of the short kernel, or one per lane
        const int gpb = lane ? sp.block_threads : short_groups_per_block(lanes, sp.block_threads);
        if (persistent) {
            int bpc = lane ? lane_max_blocks_per_cu(pen, sp.cap, cigar, sp.block_threads)
                           : short_max_blocks_per_cu(window, lanes, cigar, sp.block_threads,
                                                     sp.lds_per_block, sp.row_bytes);
            if (bpc < 1) bpc = 1;
            grid = e->num_cus * bpc;
            if (std::getenv("WFA_DEBUG"))
                std::fprintf(stderr, "libwfa plan: %s, %d threads per block, %d blocks per CU, "
                                     "%d B LDS per block\n", lane ? "lane kernel" : "short kernel",
                             sp.block_threads, bpc, sp.lds_per_block);
            const size_t needed = (N + gpb - 1) / gpb;
            if ((size_t)grid > needed) grid = (int)needed;
            // claims of several rounds keep the queue atomic off the critical
            // path; at most ~1/16 of a wave's share is claimed at once
            const size_t rounds = (N + (size_t)grid * gpb - 1) / ((size_t)grid * gpb);
            queue_chunk = (int)std::max<size_t>(1, std::min<size_t>(16, rounds / 16));
        } else {
            grid = (int)((N + gpb - 1) / gpb);
        }
    }

    if (lane && cigar)  // one history region per wavefront of the launch
        RCCHK(ws.ensure(ws.lane_hist, (size_t)grid * (sp.block_threads / 64) *
                                          lane_hist_bytes_per_wave(pen, sp.cap, true, sp.slot_cap)));
    if (lane && persistent) RCCHK(ws.ensure(ws.lane_queues, LANE_QUEUES * 32 * 4));
    flags = ws.flags.as<DevFlags>();

    // ---- device phase (graph-capturable) ----------------------------------
    // Three phases; in graph mode the first and last are captured graphs and
    // the kernel between them is launched directly, so plain events around it
    // time exactly the short-pair kernel (ev[0] start, ev[4]/ev[5] around the
    // kernel, ev[1] end).
    // pre: counters, packing, bucketing
    auto phase_pre = [&](hipStream_t q) -> int {
        // the counters, err_pair = ~0 (its two words first), the run counts,
        // the lane queues and the bucket histogram, in one launch
        static_assert(offsetof(DevFlags, err_pair) == 0, "err_pair leads DevFlags");
        FillOps fill{};
        fill.add((uint32_t*)flags, 2, ~0u);
        fill.add((uint32_t*)flags + 2, sizeof(DevFlags) / 4 - 2, 0u);
        fill.add(ws.nruns.as<uint32_t>(), N, 0u);
        if (lane && persistent) fill.add(ws.lane_queues.as<uint32_t>(), LANE_QUEUES * 32, 0u);
        if (use_short && bucket) fill.add(hist, 2 * BUCKET_KEYS, 0u);
        HIPCHK(launch_fill_multi(fill, q));
        if (ascii) {
            if (!stride_p)
                HIPCHK(launch_scan(SCAN_WORDS_P, in_pairs, N, ws.ws_p.as<uint64_t>(), ws.scan_tmp.ptr, q));
            if (!stride_t)
                HIPCHK(launch_scan(SCAN_WORDS_T, in_pairs, N, ws.ws_t.as<uint64_t>(), ws.scan_tmp.ptr, q));
            HIPCHK(launch_pack_pairs(in_pairs, N, (const uint8_t*)in_p, (const uint8_t*)in_t,
                                     stride_p ? nullptr : ws.ws_p.as<uint64_t>(),
                                     stride_t ? nullptr : ws.ws_t.as<uint64_t>(),
                                     (st.max_p + 31) / 32, (st.max_t + 31) / 32,
                                     ws.words_p.as<uint64_t>(), ws.words_t.as<uint64_t>(),
                                     ws.packed_pairs.as<PairDesc>(), &flags->err_pair, q));
        }
        if (use_short && bucket) {
            HIPCHK(launch_bucket_keys(d.pairs, N, ws.keys.as<uint32_t>(), hist, q));
            HIPCHK(launch_bucket_scatter(ws.keys.as<uint32_t>(), N, hist, taken,
                                         ws.order.as<uint32_t>(), q));
        }
        return WFA_OK;
    };
    // the short-pair kernel itself
    auto phase_kernel = [&](hipStream_t q) -> int {
        if (lane) {
            LaneArgs a{};
            a.pairs = d.pairs;
            a.pw = d.pw;
            a.tw = d.tw;
            a.order = bucket ? ws.order.as<uint32_t>() : nullptr;
            a.num = (uint32_t)N;
            a.npairs = (uint32_t)N;
            a.queue = ws.lane_queues.as<uint32_t>();
            a.pen = pen;
            a.slot_cap = sp.slot_cap;
            a.scores = d.scores;
            a.nruns = ws.nruns.as<uint32_t>();
            a.run_src = ws.run_src.as<uint64_t>();
            a.slots = ws.slots.as<uint32_t>();
            a.hist = cigar ? ws.lane_hist.as<uint32_t>() : nullptr;
            a.ovf_list = ws.ovf_list.as<uint32_t>();
            a.ovf_count = &flags->ovf_count;
            HIPCHK(launch_lane(a, sp.cap, cigar, persistent, sp.block_threads, grid, q));
        } else if (use_short) {
            ShortArgs a{};
            a.pairs = d.pairs;
            a.pw = d.pw;
            a.tw = d.tw;
            a.order = bucket ? ws.order.as<uint32_t>() : nullptr;
            a.num = (uint32_t)N;
            a.npairs = (uint32_t)N;
            a.ends = e->ends;
            a.queue = &flags->queue;
            a.queue_chunk = queue_chunk;
            a.pen = pen;
            a.cap = sp.cap;
            a.ring = sp.ring;
            a.ring2 = sp.ring2;
            a.id_off = sp.id_off;
            a.seq_words = sp.seq_words;
            a.group_bytes = sp.group_bytes;
            a.rows_bytes = sp.rows_bytes;
            a.slot_cap = sp.slot_cap;
            a.row_bytes = sp.row_bytes;
            a.scores = d.scores;
            a.nruns = ws.nruns.as<uint32_t>();
            a.run_src = ws.run_src.as<uint64_t>();
            a.slots = ws.slots.as<uint32_t>();
            a.ovf_list = ws.ovf_list.as<uint32_t>();
            a.ovf_count = &flags->ovf_count;
            HIPCHK(launch_short(a, window, lanes, cigar, persistent, sp.block_threads, grid, q));
        }
        return WFA_OK;
    };
    // post: CIGAR offsets and compaction
    auto phase_post = [&](hipStream_t q) -> int {
        if (cigar && use_short) {
            HIPCHK(launch_scan(SCAN_U32, ws.nruns.ptr, N, d.offsets, ws.scan_tmp.ptr, q));
            HIPCHK(launch_compact(ws.run_src.as<uint64_t>(),
                                  ws.slots.as<uint32_t>(), ws.slots2.as<uint32_t>(),
                                  ws.gen_runs.as<uint32_t>(), d.offsets,
                                  N, d.runs, d.capacity, &flags->total_runs, q));
        }
        return WFA_OK;
    };

    // Graph forms: 1 (default) captures the whole device phase -- counters,
    // packing, bucketing, the short-pair kernel, CIGAR offsets and
    // compaction -- as one graph, so a call is one hipGraphLaunch; 2 captures
    // the work before and after the kernel as two graphs and launches the
    // kernel between them, so that events around it time the kernel alone.
    const int form = graph ? (e->opt.use_graph == 2 ? 2 : 1) : 0;
    GraphEntry* hit = nullptr;
    if (graph) {
        GraphKey key;
        const void* ptrs[8] = {in_pairs, in_p, in_t, d.scores, d.runs, d.offsets,
                               (const void*)(uintptr_t)ws.generation, nullptr};
        for (int i = 0; i < 8; i++) key.p[i] = ptrs[i];
        key.n = N;
        key.capacity = d.capacity;
        key.form = form;
        // every value the captured launches bake in besides the pointers:
        // penalties, plan, lengths, grid, forms, free ends, queue claims
        const int ints[18] = {(int)io.enc, (int)io.mode, pen.x, pen.oe, pen.e, pen.g,
                              window * 256 + lanes, sp.cap,
                              // the packing's word counts (packed input: none)
                              ascii ? (int)st.max_p : 0, ascii ? (int)st.max_t : 0, grid,
                              (int)(bucket ? 1 : 0) | (stride_p ? 4 : 0) | (stride_t ? 8 : 0) |
                                  (persistent ? 16 : 0) | (sp.block_threads << 8),
                              e->ends.pb, e->ends.pe, e->ends.tb, e->ends.te, queue_chunk,
                              sp.slot_cap};
        for (int i = 0; i < 18; i++) key.ints[i] = ints[i];
        for (auto& g : e->graphs)
            if (g.key == key) hit = &g;
        if (!hit) {
            GraphEntry g;
            g.key = key;
            int rc;
            if (form == 1) {
                rc = capture_graph(
                    s,
                    [&](hipStream_t q) -> int {
                        RCCHK(phase_pre(q));
                        RCCHK(phase_kernel(q));
                        return phase_post(q);
                    },
                    &g.graph_all, &g.exec_all);
            } else {
                rc = capture_graph(s, phase_pre, &g.graph_pre, &g.exec_pre);
                if (rc == WFA_OK) rc = capture_graph(s, phase_post, &g.graph_post, &g.exec_post);
            }
            if (rc != WFA_OK) {
                destroy_graph(g);
                return rc;
            }
            if (e->graphs.size() >= 4) {
                destroy_graph(e->graphs.front());
                e->graphs.erase(e->graphs.begin());
            }
            e->graphs.push_back(g);
            hit = &e->graphs.back();
        }
    }
    // events: ev[0] start, ev[4] / ev[5] around the kernel (not in form 1,
    // where the kernel runs inside the graph), ev[1] end
    const double t_plan = now_ms();
    // the speculative launch stands when this plan is the one it ran
    const bool reused = spec_ent && form == 1 && hit && hit->key == spec_key;
    double t_launched = t_plan;
    if (!reused) {
        HIPCHK(hipEventRecord(e->ev[0], s));
        if (form == 1) {
            HIPCHK(hipGraphLaunch(hit->exec_all, s));
        } else {
            if (hit) HIPCHK(hipGraphLaunch(hit->exec_pre, s)); else RCCHK(phase_pre(s));
            HIPCHK(hipEventRecord(e->ev[4], s));
            RCCHK(phase_kernel(s));
            HIPCHK(hipEventRecord(e->ev[5], s));
            if (hit) HIPCHK(hipGraphLaunch(hit->exec_post, s)); else RCCHK(phase_post(s));
        }
        HIPCHK(hipEventRecord(e->ev[1], s));
        // the run total of the short kernel's pairs (written by the
        // compaction into total_runs) comes back with the flags
        HIPCHK(hipMemcpyAsync(rb, flags, sizeof(DevFlags), hipMemcpyDeviceToHost, s));
        t_launched = now_ms();
        HIPCHK(hipStreamSynchronize(s));
    }
    if (form == 1) {  // the next call with the same buffers and settings may start this graph early
        e->spec.valid = true;
        e->spec.key = hit->key;
        e->spec.opt = e->opt;
        e->spec.ends = e->ends;
        e->spec.heur = e->heur;
    }
    const double t_flags = now_ms();
    DevFlags fl;
    uint64_t short_total = 0;
    std::memcpy(&fl, rb, sizeof(fl));
    if (cigar && use_short) short_total = fl.total_runs;
    if (fl.err_pair != ~0ull) {
        if (bad_pair) *bad_pair = (int64_t)fl.err_pair;
        return WFA_E_ALPHABET;
    }

    // ---- the cascade: wider short-kernel passes (windows 64, 128, 256 above
    // the first, up to the cascade's largest), each over the pairs the
    // previous pass handed over, before anything goes to the general kernel ---
    uint64_t general_done = 0, requeued = 0, gen_used = 0;
    uint32_t ovf_final = use_short ? fl.ovf_count : 0;
    const Buf* ovf_buf = &ws.ovf_list;
    int window2 = 0;
    double ms_cascade = 0.0;
    if (use_short) requeued += fl.ovf_count;
    if (use_short && fl.ovf_count > 0 && e->opt.cascade_window >= 0) {
        const int wmax = e->opt.cascade_window > 0 ? e->opt.cascade_window : 256;
        RCCHK(ws.ensure(ws.ovf_list2, (size_t)fl.ovf_count * 4));
        Buf* lists[2] = {&ws.ovf_list, &ws.ovf_list2};
        int in_list = 0;
        uint64_t slots2_used = 0;  // words of slots2 taken by earlier passes
        // the cascade's windows: 64, 128, 256 above the first window
        for (int w2 = 64; w2 <= wmax && ovf_final > 0; w2 *= 2) {
            if (w2 <= window) continue;
            const int l2 = default_lanes(w2);
            ShortPlan sp2;
            if (!short_shape_supported(w2, l2) ||
                short_plan(e, pen, cigar, w2, l2, default_cap(pen, w2), max_len, &sp2) != WFA_OK)
                break;
            const uint32_t n2 = ovf_final;
            if (cigar)
                RCCHK(ws.grow_keep(ws.slots2, (slots2_used + (uint64_t)n2 * sp2.slot_cap) * 4,
                                   slots2_used * 4, s));
            const int gpb2 = short_groups_per_block(l2, sp2.block_threads);
            int bpc2 = short_max_blocks_per_cu(w2, l2, cigar, sp2.block_threads,
                                               sp2.lds_per_block, sp2.row_bytes);
            if (bpc2 < 1) bpc2 = 1;
            int grid2 = e->num_cus * bpc2;
            const size_t need2 = (n2 + gpb2 - 1) / gpb2;
            if ((size_t)grid2 > need2) grid2 = (int)need2;
            ShortArgs a{};
            a.pairs = d.pairs;
            a.pw = d.pw;
            a.tw = d.tw;
            a.order = lists[in_list]->as<uint32_t>();  // the previous pass's hand-overs
            a.num = n2;
            a.npairs = (uint32_t)N;
            a.ends = e->ends;
            a.queue = &flags->queue2;
            a.queue_chunk = 1;
            a.pen = pen;
            a.cap = sp2.cap;
            a.ring = sp2.ring;
            a.ring2 = sp2.ring2;
            a.id_off = sp2.id_off;
            a.seq_words = sp2.seq_words;
            a.group_bytes = sp2.group_bytes;
            a.rows_bytes = sp2.rows_bytes;
            a.slot_cap = sp2.slot_cap;
            a.row_bytes = sp2.row_bytes;
            a.scores = d.scores;
            a.nruns = ws.nruns.as<uint32_t>();
            a.run_src = ws.run_src.as<uint64_t>();
            a.run_src_add = SLOTS2_BIT + slots2_used;
            a.slots = cigar ? ws.slots2.as<uint32_t>() + slots2_used : nullptr;
            a.ovf_list = lists[1 - in_list]->as<uint32_t>();
            a.ovf_count = &flags->ovf_count2;
            HIPCHK(launch_fill_u32(&flags->ovf_count2, 0u, 2, s));  // ovf_count2, queue2
            HIPCHK(hipEventRecord(e->ev[10], s));
            HIPCHK(launch_short(a, w2, l2, cigar, true, sp2.block_threads, grid2, s));
            HIPCHK(hipEventRecord(e->ev[11], s));
            uint32_t n_out = 0;
            HIPCHK(hipMemcpyAsync(&n_out, &flags->ovf_count2, 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            ms_cascade += ev_ms(e->ev[10], e->ev[11]);
            if (cigar) slots2_used += (uint64_t)n2 * sp2.slot_cap;
            ovf_final = n_out;
            in_list = 1 - in_list;
            ovf_buf = lists[in_list];
            window2 = w2;
            requeued += n_out;
        }
    }

    // ---- general kernel for the rest ---------------------------------------
    std::vector<uint32_t> pending;
    if (!use_short) {
        pending.resize(N);
        for (size_t i = 0; i < N; i++) pending[i] = (uint32_t)i;
    } else if (ovf_final) {
        pending.resize(ovf_final);
        HIPCHK(hipMemcpy(pending.data(), ovf_buf->ptr, ovf_final * 4ull, hipMemcpyDeviceToHost));
        std::sort(pending.begin(), pending.end());
    }
    // the common case ends here: the first pass held every pair and its
    // offsets and runs are written, so nothing more runs on the device
    const bool tail = !pending.empty() || !use_short || fl.ovf_count > 0;
    if (tail) HIPCHK(hipEventRecord(e->ev[2], s));
    if (!pending.empty()) {
        int64_t gave_up = -1;
        const int rg = run_general(e, pen, cigar, d, st, pending, gen_used, s, &general_done,
                                   &requeued, &gave_up);
        if (rg == WFA_E_LIMIT && bad_pair) *bad_pair = gave_up;
        if (rg != WFA_OK) {
            (void)finish_user();
            return rg;
        }
        flags = ws.flags.as<DevFlags>();
    }
    if (tail) HIPCHK(hipEventRecord(e->ev[3], s));

    // ---- CIGAR offsets and compaction ------------------------------------------
    uint64_t total = 0;
    if (cigar) {
        // any hand-over changes run counts after the first pass's scan
        const bool rescan = !use_short || fl.ovf_count > 0;
        if (rescan) {
            RCCHK(ws.ensure(ws.scan_tmp, scan_temp_bytes(N + 1) + 64));
            HIPCHK(launch_scan(SCAN_U32, ws.nruns.ptr, N, d.offsets, ws.scan_tmp.ptr, s));
            HIPCHK(hipMemcpyAsync(&total, d.offsets + N, 8, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        } else {
            total = short_total;
        }
        if (rescan && total <= d.capacity)
            HIPCHK(launch_compact(ws.run_src.as<uint64_t>(),
                                  ws.slots.as<uint32_t>(), ws.slots2.as<uint32_t>(),
                                  ws.gen_runs.as<uint32_t>(), d.offsets, N,
                                  d.runs, d.capacity, nullptr, s));
        if (cigar_needed) *cigar_needed = (size_t)total;
    }
    if (tail) HIPCHK(hipEventRecord(e->ev[8], s));
    RCCHK(finish_user(!tail));

    wfa_stats& L = e->last;
    L.pairs = N;
    L.general_pairs = general_done;
    L.short_pairs = use_short ? N - ovf_final : 0;
    L.cascade_window = window2;
    L.requeued = requeued;
    L.cigar_runs = total;
    L.window = use_short && !lane ? window : 0;
    L.lanes_per_pair = use_short ? lanes : 0;
    L.lane_kernel = lane ? 1 : 0;
    L.step_cap = use_short ? sp.cap : 0;
    L.schedule = !use_short ? WFA_SCHED_GENERAL : (persistent ? WFA_SCHED_PERSISTENT : WFA_SCHED_PLAIN);
    L.graph_replayed = form;
    const double ms_tail = tail ? ev_ms(e->ev[3], e->ev[8]) : 0.0;
    if (form == 1) {  // the whole first pass ran as one graph
        L.ms_pack = 0.0;
        L.ms_align = ev_ms(e->ev[0], e->ev[1]) + ms_cascade;
        L.ms_compact = ms_tail;
    } else {
        L.ms_pack = use_short ? ev_ms(e->ev[0], e->ev[4]) : 0.0;
        L.ms_align = (use_short ? ev_ms(e->ev[4], e->ev[5]) : 0.0) + ms_cascade;
        L.ms_compact = (use_short ? ev_ms(e->ev[5], e->ev[1]) : 0.0) + ms_tail;
    }
    L.ms_general = tail ? ev_ms(e->ev[2], e->ev[3]) : 0.0;
    L.ms_total = now_ms() - t_start;
    if (debug_level() >= 2)
        std::fprintf(stderr, "libwfa call: %d pairs, host ms: stats %.3f, plan %.3f, launch %.3f, "
                             "wait %.3f, rest %.3f, total %.3f (device first pass %.3f)\n",
                     (int)N, t_stats - t_start, t_plan - t_stats, t_launched - t_plan,
                     t_flags - t_launched, now_ms() - t_flags, L.ms_total, L.ms_align);

    e->last_valid = cigar;
    e->last_n = N;
    e->last_mem = io.mem;
    e->last_total = total;
    if (cigar && total > io.capacity) return WFA_E_CAPACITY;
    return WFA_OK;
}
