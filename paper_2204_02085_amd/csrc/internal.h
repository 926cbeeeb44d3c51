// Library-internal state: device workspace, plans, engines and contexts.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <memory>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "../../include/wfa.h"
#include "kernels.h"

struct Buf {
    void* ptr = nullptr;
    size_t bytes = 0;
    template <class T>
    T* as() const {
        return (T*)ptr;
    }
};

// Device buffers of one engine.  Each grows on demand; the sum stays within
// `budget` bytes (WFA_E_NOMEM otherwise).
struct Workspace {
    size_t budget = 0;
    size_t total = 0;
    uint64_t generation = 0;  // bumped whenever a buffer moves (invalidates graphs)
    // planning / packing
    Buf stats, flags, scan_tmp, ws_p, ws_t, words_p, words_t, packed_pairs;
    // host-memory pipeline: device copies of the whole batch's inputs and
    // outputs (host_off: offsets of the batch, host_loff: of one chunk)
    Buf in_pairs, in_p, in_t, out_scores, out_runs, out_offsets, host_off, host_loff;
    // short kernel (slots2 / ovf_list2: the wider second pass)
    Buf nruns, run_src, slots, ovf_list, order, keys, hist, slots2, ovf_list2;
    // general kernel
    Buf jobs, job_nruns, job_offsets, fail_list, arena, gen_runs, gen_tmp, job_used, gen_state,
        gen_slices;
    // one-pair-per-lane kernel: CIGAR history of every wavefront of a launch,
    // and the claim counters of its persistent form
    Buf lane_hist, lane_queues;
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
    // the owning engine's streams: buffers are allocated and freed in stream
    // order on the first one once all of them have drained, so growing one
    // engine's buffers never waits for work of other engines on the device
    hipStream_t own[3] = {nullptr, nullptr, nullptr};
    // Fixed mode (the allocation-free entry point): every buffer is carved
    // from one caller-provided device region by a bump pointer and nothing is
    // ever allocated; a buffer that does not fit is WFA_E_NOMEM.  Releasing
    // the most recently carved buffer hands its bytes back.
    unsigned char* fixed_base = nullptr;
    size_t fixed_size = 0, fixed_top = 0;
    void use_fixed(void* base, size_t size);  // start carving from an empty region

    std::array<Buf*, 37> all() {
        return {&stats,   &flags,      &scan_tmp, &ws_p,        &ws_t,      &words_p,
                &words_t, &packed_pairs, &in_pairs, &in_p,      &in_t,      &out_scores,
                &out_runs, &out_offsets, &host_off, &host_loff, &nruns,   &run_src,
                &slots,   &ovf_list,   &order,    &keys,        &hist,      &slots2,
                &ovf_list2, &jobs,     &job_nruns, &job_offsets, &fail_list, &arena,
                &gen_runs, &gen_tmp, &job_used, &gen_state, &gen_slices, &lane_hist,
                &lane_queues};
    }
    int ensure(Buf& b, size_t bytes);
    // grow to at least `bytes`, keeping the first `keep` bytes (copied on `s`,
    // which is synchronised before the old block is freed)
    int grow_keep(Buf& b, size_t bytes, size_t keep, hipStream_t s);
    void release(Buf& b);
    void release_all();
    int ensure_pinned(size_t bytes);
};

// Device-side flags read back once per batch.
struct DevFlags {
    unsigned long long err_pair;  // first pair with a non-ACGT byte (~0: none)
    uint32_t ovf_count;           // pairs the short kernel handed over
    uint32_t queue;               // persistent queue head
    uint32_t fail_count;          // general jobs whose slice was too small
    uint32_t ovf_count2;          // pairs a cascade pass (a wider short pass) handed over
    uint32_t queue2;              // queue head of a cascade pass
    uint32_t pad;
    uint64_t total_runs;          // run total of the first pass (written by the compaction)
    unsigned long long gave_up;   // first pair the general kernel gave up on (~0: none)
};

struct ShortPlan {
    int window = 0, lanes = 32, cap = 0, seq_words = 0, ring = 0, group_bytes = 0, slot_cap = 0;
    int rows_bytes = 0, ring2 = 0, id_off = 0;
    int row_bytes = 2;
    int block_threads = 256, lds_per_block = 0;
};

// Everything a captured graph bakes in: buffer addresses, sizes, the plan
// and the caller's full CIGAR capacity (compaction writes nothing when the
// runs exceed it, so a replay under another capacity would be wrong).
struct GraphKey {
    const void* p[8] = {};
    size_t n = 0;
    uint64_t capacity = 0;
    int form = 0;  // 1: one graph of the whole device phase, 2: pre / post graphs
    int ints[18] = {};
    bool operator==(const GraphKey& o) const;
};

// Captured graphs of one plan.  Form 1: one graph holding the work before
// the short-pair kernel (counters, packing, bucketing), the kernel and the
// work after it (CIGAR offsets, compaction).  Form 2: the work before and
// after the kernel as two graphs, the kernel launched between them, so that
// events recorded around it time the kernel alone.
struct GraphEntry {
    GraphKey key;
    hipGraph_t graph_all = nullptr, graph_pre = nullptr, graph_post = nullptr;
    hipGraphExec_t exec_all = nullptr, exec_pre = nullptr, exec_post = nullptr;
};

// Everything one batch needs: a stream, a workspace, events and options.
struct Engine {
    int device = 0;
    int num_cus = 256;
    hipStream_t stream = nullptr;
    hipStream_t h2d = nullptr, d2h = nullptr;  // copy streams of the host-memory pipeline
    Workspace ws;
    hipEvent_t ev[12] = {};
    wfa_options opt{};
    wfa::Ends ends{};  // free ends of later calls (all zero: global alignment)
    wfa::Heuristic heur{};  // WF-adaptive heuristic of later calls (mwl 0: exact)
    // page-locked landing slots for the device path's small read-backs (batch
    // facts, flags and run total), so those copies are asynchronous and one
    // stream synchronisation ends each round trip
    void* readback = nullptr;
    // The last call's whole-pass graph and what it was planned under: a call
    // with the same buffers, sizes, packed input and settings launches that
    // graph right behind the batch-facts kernel, before the facts are back,
    // and keeps its results when the facts lead to the same plan (any plan
    // aligns any batch exactly; only its speed depends on the facts).
    struct Spec {
        bool valid = false;
        GraphKey key;
        wfa_options opt{};
        wfa::Ends ends{};
        wfa::Heuristic heur{};
    } spec;
    wfa_stats last{};
    std::vector<GraphEntry> graphs;
    // state kept for wfa_copy_last_cigars
    bool last_valid = false;
    size_t last_n = 0;
    int last_mem = 0;
    uint64_t last_total = 0;
};

// The context's own engine, plus the engines of closed servers: a server
// opened later takes them over with their streams and device buffers
// instead of allocating its own again.  `fixed` serves the allocation-free
// entry point: its workspace lives in the device's static scratch array.
struct wfa_ctx : Engine {
    std::mutex idle_mu;
    std::vector<std::unique_ptr<Engine>> idle;
    std::unique_ptr<Engine> fixed;
};

// Diagnostics level from WFA_DEBUG (unset or 0: none; 1: plans and passes;
// 2: also host time per phase of every device-path call), read once.
inline int debug_level() {
    static const int level = [] {
        const char* v = std::getenv("WFA_DEBUG");
        return v ? std::max(1, std::atoi(v)) : 0;
    }();
    return level;
}

// Allocation-free entry point: the device address of the static scratch
// array (resolved once per device at context creation) and its size.
int noalloc_setup(int device);
void* noalloc_scratch(int device);
size_t noalloc_scratch_bytes();

// Batch inputs/outputs as given by the caller.
struct BatchIO {
    const void* patterns;
    const void* texts;
    const wfa_pair* pairs;
    size_t n;
    wfa_encoding enc;
    wfa_memspace mem;
    wfa_penalties pen;
    wfa_mode mode;
    int32_t* scores;
    uint32_t* runs;
    size_t capacity;
    uint64_t* offsets;
    bool no_graph = false;  // never capture or replay graphs for this call
};

int make_pen(const wfa_penalties& p, wfa::Pen* out);
int default_cap(const wfa::Pen& pen, int window);
int default_lanes(int window);
int short_plan(Engine* ctx, const wfa::Pen& pen, bool cigar, int window, int lanes, int cap,
               uint32_t max_len, ShortPlan* sp);
// Any batch: device memory directly, host memory through the chunk pipeline.
int engine_align(Engine* e, const BatchIO& io, hipStream_t user_stream, size_t* cigar_needed,
                 int64_t* bad_pair);
int engine_align_device(Engine* e, const BatchIO& io, hipStream_t user_stream,
                        size_t* cigar_needed, int64_t* bad_pair);
int engine_align_host(Engine* e, const BatchIO& io, hipStream_t user_stream, size_t* cigar_needed,
                      int64_t* bad_pair);
void graph_cache_clear(Engine* e);
int engine_init(Engine* e, int device, size_t budget);
void engine_destroy(Engine* e);
void destroy_graph(GraphEntry& g);
