// Allocation-free variant of wfa_align_batch, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// Its device workspace -- batch statistics, flags and counters, packed
// sequences, per-pair run counts and sources, CIGAR slots, bucketing keys
// and permutation, the cascade's slots and the general kernel's arena -- is
// carved from one file-scope device array, `scratch`, by a bump pointer.
// Each GPU the library runs on holds its own copy of the array from the time
// the library's code object is loaded there until the process ends.  Its
// device address is resolved once per device, at context creation, with that
// device current; host code passes that address (never the array's name,
// which is a host-side stand-in) to the kernels.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/wfa.h"
#include "internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[WFA_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_addr[MAX_DEVICES] = {};

}  // namespace

int noalloc_setup(int device) {
    if (device < 0 || device >= MAX_DEVICES) return WFA_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_addr[device]) return WFA_OK;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) {
        (void)hipGetLastError();
        return WFA_E_DEVICE;
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    (void)hipSetDevice(prev);
    if (e != hipSuccess || !p) {
        std::fprintf(stderr, "libwfa: hipGetSymbolAddress(scratch) on device %d: %s\n", device,
                     hipGetErrorString(e));
        (void)hipGetLastError();
        return WFA_E_DEVICE;
    }
    g_addr[device] = p;
    return WFA_OK;
}

void* noalloc_scratch(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_addr[device];
}

size_t noalloc_scratch_bytes() { return WFA_NOALLOC_SCRATCH_BYTES; }

extern "C" int wfa_align_batch_noalloc(wfa_ctx* ctx, const void* patterns, const void* texts,
                                       const wfa_pair* pairs, size_t num_pairs, wfa_encoding enc,
                                       wfa_penalties pen, wfa_mode mode, int32_t* scores,
                                       uint32_t* cigar_runs, size_t cigar_capacity,
                                       uint64_t* cigar_offsets, size_t* cigar_needed,
                                       int64_t* bad_pair, void* stream) {
    if (bad_pair) *bad_pair = -1;
    if (cigar_needed) *cigar_needed = 0;
    if (!ctx || !ctx->fixed) return WFA_E_INVAL;
    if (num_pairs > WFA_NOALLOC_MAX_PAIRS) {
        std::fprintf(stderr, "libwfa: wfa_align_batch_noalloc takes at most %u pairs per call "
                             "(got %zu)\n", (unsigned)WFA_NOALLOC_MAX_PAIRS, num_pairs);
        return WFA_E_INVAL;
    }
    void* base = noalloc_scratch(ctx->device);
    if (!base) return WFA_E_DEVICE;
    Engine* e = ctx->fixed.get();
    e->opt = ctx->opt;
    e->ends = ctx->ends;
    e->heur = ctx->heur;
    // every call starts from an empty region; the kernels clear the flags,
    // counters and run counts they rely on before using them
    e->ws.use_fixed(base, WFA_NOALLOC_SCRATCH_BYTES);
    BatchIO io{patterns, texts, pairs, num_pairs, enc, WFA_DEVICE, pen, mode,
               scores, cigar_runs, cigar_capacity, cigar_offsets};
    io.no_graph = true;  // capturing a graph may allocate
    return engine_align_device(e, io, (hipStream_t)stream, cigar_needed, bad_pair);
}
