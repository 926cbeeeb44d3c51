// Autotuner: picks the short-kernel window (lane groups per wavefront and
// diagonals per lane), step cap (LDS rows per pair), workgroup size, schedule
// and bucketing for a class of batches by timing candidates on a sample of
// the batch.  Every candidate must return byte-identical scores and CIGARs;
// the winner is cached in a small JSON file keyed by device architecture and
// workload class.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/wfa.h"
#include "internal.h"

namespace {

struct Candidate {
    wfa_options opt;
    double ms = 1e30;
};

std::string class_key(const char* arch, const wfa_penalties& pen, int mode, uint32_t max_len,
                      uint32_t max_diff, size_t n, const wfa::Ends& ends,
                      const wfa::Heuristic& heur) {
    // length and length-difference classes on a log2 scale
    auto lg = [](uint32_t v) { return v ? 32 - __builtin_clz(v) : 0; };
    std::ostringstream k;
    k << arch << "/x" << pen.mismatch << "o" << pen.gap_open << "e" << pen.gap_extend << "/"
      << (mode == WFA_CIGAR ? "cigar" : "score") << "/len" << lg(max_len) << "/diff" << lg(max_diff)
      << "/n" << lg((uint32_t)std::min<size_t>(n, 1u << 30));
    if (ends.pb || ends.pe || ends.tb || ends.te)  // ends-free: the free ends' classes
        k << "/ends" << lg(std::min<uint32_t>(ends.pb, max_len)) << "."
          << lg(std::min<uint32_t>(ends.pe, max_len)) << "." << lg(std::min<uint32_t>(ends.tb, max_len))
          << "." << lg(std::min<uint32_t>(ends.te, max_len));
    if (heur.mwl > 0) k << "/adaptive" << heur.mwl << "." << heur.mdt;
    return k.str();
}

bool load_entry(const char* path, const std::string& key, wfa_options* out) {
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    const std::string needle = "\"" + key + "\"";
    while (std::getline(f, line)) {
        if (line.find(needle) == std::string::npos) continue;
        wfa_options o{};
        auto get = [&](const char* name) -> int {
            const std::string t = std::string("\"") + name + "\": ";
            const size_t p = line.find(t);
            return p == std::string::npos ? 0 : std::atoi(line.c_str() + p + t.size());
        };
        o.schedule = get("schedule");
        o.window = get("window");
        o.lanes_per_pair = get("lanes_per_pair");
        o.step_cap = get("step_cap");
        o.block_threads = get("block_threads");
        o.bucket = get("bucket");
        o.use_graph = get("use_graph");
        o.lane_kernel = get("lane_kernel");
        *out = o;
        return true;
    }
    return false;
}

void store_entry(const char* path, const std::string& key, const Candidate& c) {
    if (!path) return;
    std::vector<std::string> lines;
    {
        std::ifstream f(path);
        std::string line;
        const std::string needle = "\"" + key + "\"";
        while (std::getline(f, line))
            if (line.size() > 2 && line.find(needle) == std::string::npos && line[0] == ' ')
                lines.push_back(line);
    }
    std::ostringstream e;
    e << "  \"" << key << "\": {\"schedule\": " << c.opt.schedule << ", \"window\": " << c.opt.window
      << ", \"lanes_per_pair\": " << c.opt.lanes_per_pair
      << ", \"step_cap\": " << c.opt.step_cap << ", \"block_threads\": " << c.opt.block_threads
      << ", \"bucket\": " << c.opt.bucket << ", \"use_graph\": " << c.opt.use_graph
      << ", \"lane_kernel\": " << c.opt.lane_kernel
      << ", \"ms_per_million_pairs\": " << c.ms << "}";
    lines.push_back(e.str());
    std::ofstream f(path, std::ios::trunc);
    f << "{\n";
    for (size_t i = 0; i < lines.size(); i++) {
        std::string l = lines[i];
        while (!l.empty() && (l.back() == ',' || l.back() == ' ')) l.pop_back();
        f << l << (i + 1 < lines.size() ? ",\n" : "\n");
    }
    f << "}\n";
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace

extern "C" int wfa_autotune(wfa_ctx* ctx, const void* patterns, const void* texts,
                            const wfa_pair* pairs, size_t num_pairs, wfa_encoding enc,
                            wfa_memspace mem, wfa_penalties pen, wfa_mode mode,
                            size_t sample_pairs, const char* cache_path, int force,
                            wfa_options* chosen) {
    if (!ctx || !chosen || !num_pairs || !pairs) return WFA_E_INVAL;
    wfa::Pen P;
    if (make_pen(pen, &P) != WFA_OK) return WFA_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return WFA_E_DEVICE;
    const size_t n = std::min(num_pairs, sample_pairs ? sample_pairs : (size_t)262144);
    const bool cigar = mode == WFA_CIGAR;

    // lengths of the sample (descriptors may live on the device)
    std::vector<wfa_pair> host_pairs(n);
    if (mem == WFA_DEVICE) {
        if (hipMemcpy(host_pairs.data(), pairs, n * sizeof(wfa_pair), hipMemcpyDeviceToHost) !=
            hipSuccess)
            return WFA_E_DEVICE;
    } else {
        std::memcpy(host_pairs.data(), pairs, n * sizeof(wfa_pair));
    }
    uint32_t max_len = 0, max_diff = 0;
    for (auto& q : host_pairs) {
        max_len = std::max(max_len, std::max(q.p_len, q.t_len));
        max_diff = std::max(max_diff, q.p_len > q.t_len ? q.p_len - q.t_len : q.t_len - q.p_len);
    }
    hipDeviceProp_t prop;
    const char* arch = "gfx";
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
    std::string a(arch);
    a = a.substr(0, a.find(':'));
    const std::string key = class_key(a.c_str(), pen, mode, max_len, max_diff, num_pairs, ctx->ends,
                                        ctx->heur);
    if (!force && load_entry(cache_path, key, chosen)) {
        ctx->opt = *chosen;
        return WFA_OK;
    }

    // outputs of the sample (device)
    Workspace tmp;
    tmp.budget = (size_t)16 << 30;
    Buf d_scores, d_runs, d_off;
    const size_t cap = cigar ? n * 64 + 1024 : 1;
    int rc = tmp.ensure(d_scores, n * 4);
    if (rc == WFA_OK) rc = tmp.ensure(d_runs, cap * 4);
    if (rc == WFA_OK) rc = tmp.ensure(d_off, (n + 1) * 8);
    if (rc != WFA_OK) {
        tmp.release_all();
        return rc;
    }
    std::vector<int32_t> ref_scores, scores(n);
    const wfa_options saved = ctx->opt;

    // Largest score step of the sample (a score-only pass with the default
    // options): step caps just above it keep the LDS per pair small without
    // sending the sample's pairs to the general kernel.
    int sample_steps = -1;
    {
        ctx->opt = wfa_options{};
        BatchIO io{patterns, texts, pairs, n, enc, mem, pen, WFA_SCORE,
                   mem == WFA_DEVICE ? d_scores.as<int32_t>() : scores.data(), nullptr, 0, nullptr};
        size_t needed = 0;
        int64_t bad = -1;
        rc = engine_align(ctx, io, nullptr, &needed, &bad);
        ctx->opt = saved;
        if (rc != WFA_OK) {
            tmp.release_all();
            return rc;
        }
        if (mem == WFA_DEVICE &&
            hipMemcpy(scores.data(), d_scores.ptr, n * 4, hipMemcpyDeviceToHost) != hipSuccess) {
            tmp.release_all();
            return WFA_E_DEVICE;
        }
        for (int32_t v : scores) sample_steps = std::max(sample_steps, v / P.g);
    }

    std::vector<uint64_t> ref_off, off(n + 1);
    std::vector<uint32_t> ref_runs, runs;
    Candidate best;
    int status = WFA_OK;

    // Times one candidate (fastest of `reps` calls after a warm-up call) and
    // checks that its results equal the first candidate's.  Returns WFA_OK,
    // WFA_E_NOMEM for a candidate that does not fit (skipped), or an error.
    auto evaluate = [&](Candidate& c, int reps) -> int {
        ctx->opt = c.opt;
        BatchIO io{patterns, texts, pairs, n, enc, mem, pen, mode,
                   mem == WFA_DEVICE ? d_scores.as<int32_t>() : scores.data(),
                   nullptr, 0, nullptr};
        std::vector<uint32_t> hruns;
        if (mem == WFA_DEVICE) {
            io.runs = cigar ? d_runs.as<uint32_t>() : nullptr;
            io.capacity = cigar ? cap : 0;
            io.offsets = cigar ? d_off.as<uint64_t>() : nullptr;
        } else {
            hruns.resize(cap);
            io.runs = cigar ? hruns.data() : nullptr;
            io.capacity = cigar ? cap : 0;
            io.offsets = cigar ? off.data() : nullptr;
        }
        size_t needed = 0;
        int64_t bad = -1;
        int r = engine_align(ctx, io, nullptr, &needed, &bad);  // warm-up (plans, graphs)
        if (r != WFA_OK) return r;
        double bestrep = 1e30;
        for (int k = 0; k < reps; k++) {
            const double t0 = now_ms();
            r = engine_align(ctx, io, nullptr, &needed, &bad);  // synchronous
            const double t1 = now_ms();
            if (r != WFA_OK) return r == WFA_E_NOMEM ? WFA_E_DEVICE : r;
            bestrep = std::min(bestrep, t1 - t0);
        }
        c.ms = bestrep / (double)n * 1e6;
        // results of every candidate must be identical
        if (mem == WFA_DEVICE) {
            (void)hipMemcpy(scores.data(), d_scores.ptr, n * 4, hipMemcpyDeviceToHost);
            if (cigar) {
                (void)hipMemcpy(off.data(), d_off.ptr, (n + 1) * 8, hipMemcpyDeviceToHost);
                runs.resize(off[n]);
                if (off[n])
                    (void)hipMemcpy(runs.data(), d_runs.ptr, off[n] * 4, hipMemcpyDeviceToHost);
            }
        } else if (cigar) {
            runs.assign(hruns.begin(), hruns.begin() + off[n]);
        }
        if (ref_scores.empty()) {
            ref_scores = scores;
            ref_off = off;
            ref_runs = runs;
        } else if (scores != ref_scores || (cigar && (off != ref_off || runs != ref_runs))) {
            std::fprintf(stderr, "libwfa autotune: candidate window=%d lanes=%d cap=%d bt=%d "
                                 "sched=%d changed the results\n",
                         c.opt.window, c.opt.lanes_per_pair, c.opt.step_cap, c.opt.block_threads,
                         c.opt.schedule);
            return WFA_E_DEVICE;
        }
        if (c.ms < best.ms) best = c;
        return WFA_OK;
    };

    // Stage 1: every short-kernel shape (window, lanes per pair) whose window
    // can hold the target diagonal, plain schedule, and the general kernel.
    struct Shape {
        int w, g, cap0, caps;
        double ms;
    };
    std::vector<Shape> shapes;
    // the one-pair-per-lane kernel (window 0 in the shape list): step cap 16,
    // or 8 when the sample's largest score step allows
    if (wfa::lane_supported(P, 16, max_len) && ctx->ends.pb == 0 && ctx->ends.pe == 0 &&
        ctx->ends.tb == 0 && ctx->ends.te == 0) {
        const int lc = (sample_steps >= 0 && sample_steps <= 8) ? 8 : 16;
        shapes.push_back({0, 1, 16, lc, 1e30});
    }
    const int windows[] = {16, 24, 32, 48, 64, 128, 256};
    for (int w : windows) {
        if (w < 2 * (int)max_diff + 4 && w != 256) continue;  // the target must fit the window
        const int cap0 = default_cap(P, w);
        const int caps = (sample_steps >= 0 && sample_steps < cap0)
                             ? std::max(sample_steps, 1)
                             : std::max(P.oe + P.x, cap0 * 2 / 3);
        for (int g : {8, 16, 32, 64})
            if (wfa::short_shape_supported(w, g)) shapes.push_back({w, g, cap0, caps, 1e30});
    }
    for (auto& sh : shapes) {
        Candidate c{};
        c.opt.schedule = WFA_SCHED_PLAIN;
        c.opt.window = sh.w;
        c.opt.lanes_per_pair = sh.w ? sh.g : 0;
        c.opt.step_cap = sh.caps;
        c.opt.block_threads = sh.w ? 128 : 256;
        c.opt.bucket = -1;
        c.opt.use_graph = -1;
        c.opt.lane_kernel = sh.w ? -1 : 1;
        const int r = evaluate(c, 3);
        if (r == WFA_OK) sh.ms = c.ms;
        else if (r != WFA_E_NOMEM) { status = r; break; }
    }
    if (status == WFA_OK) {
        Candidate g{};
        g.opt.schedule = WFA_SCHED_GENERAL;
        g.opt.use_graph = -1;
        const int r = evaluate(g, 1);
        if (r != WFA_OK && r != WFA_E_NOMEM) status = r;
    }
    if (status == WFA_OK) {  // the library's own per-batch choice is always a candidate
        Candidate dflt{};
        const int r = evaluate(dflt, 5);
        if (r != WFA_OK && r != WFA_E_NOMEM) status = r;
    }
    // Stage 2: the two fastest shapes, every workgroup size, schedule form
    // (plain; persistent with and without bucketing) and step cap.
    std::sort(shapes.begin(), shapes.end(), [](const Shape& a, const Shape& b) { return a.ms < b.ms; });
    for (size_t i = 0; i < shapes.size() && i < 2 && status == WFA_OK; i++) {
        const Shape& sh = shapes[i];
        if (sh.ms >= 1e30) break;
        for (int bt : {64, 128, 256}) {
            for (int form : {0, 1, 2}) {
                for (int capx : {sh.caps, sh.cap0}) {
                    if (capx == sh.cap0 && sh.cap0 == sh.caps) continue;
                    Candidate c{};
                    c.opt.schedule = form == 0 ? WFA_SCHED_PLAIN : WFA_SCHED_PERSISTENT;
                    c.opt.window = sh.w;
                    c.opt.lanes_per_pair = sh.w ? sh.g : 0;
                    c.opt.lane_kernel = sh.w ? -1 : 1;
                    c.opt.step_cap = capx;
                    c.opt.block_threads = bt;
                    c.opt.bucket = form == 1 ? 1 : -1;
                    c.opt.use_graph = 1;  // pre/post phases replayed in every form
                    const int r = evaluate(c, 5);
                    if (r != WFA_OK && r != WFA_E_NOMEM) {
                        status = r;
                        break;
                    }
                }
                if (status != WFA_OK) break;
            }
            if (status != WFA_OK) break;
        }
    }
    tmp.release_all();
    if (status != WFA_OK || best.ms >= 1e30) {
        ctx->opt = saved;
        return status != WFA_OK ? status : WFA_E_NOMEM;
    }
    *chosen = best.opt;
    ctx->opt = best.opt;
    store_entry(cache_path, key, best);
    return WFA_OK;
}
