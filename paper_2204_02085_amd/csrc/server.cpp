// Serving: continuous batching of alignment requests over several streams.
//
// Requests are copied on submit and queued in arrival order.  Each worker
// owns one engine (stream + device workspace).  Whenever a worker is free it
// forms a batch from the head of the queue -- the unadmitted remainder of
// the oldest request first, then later requests -- up to max_chunk_pairs
// pairs and within the memory budget, reserves the batch's estimated device
// bytes, runs it, releases the reservation and hands every pair's result
// back to its request.  Several workers run batches at once on their own
// streams, so work of different requests overlaps on the device.  Pairs are
// aligned independently, so a request's results do not depend on which batch
// its pairs rode in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "../../include/wfa.h"
#include "internal.h"

namespace {

struct Piece {
    uint64_t ticket;
    size_t first, count;
};

struct Request {
    uint64_t ticket = 0;
    std::vector<uint8_t> pat, txt;
    std::vector<wfa_pair> pairs;   // byte offsets into pat / txt
    std::vector<size_t> est_prefix;  // estimated bytes of pairs [0, i)
    size_t next = 0;               // first pair not yet admitted
    size_t done_pairs = 0;
    int status = WFA_OK;
    double t_submit = 0, t_admit = -1, t_done = -1;
    // results, assembled as pieces finish
    std::vector<int32_t> scores;
    std::map<size_t, std::vector<uint32_t>> piece_runs;     // first -> runs
    std::map<size_t, std::vector<uint32_t>> piece_counts;   // first -> runs per pair
    std::vector<uint32_t> runs;
    std::vector<uint64_t> offsets;
    bool finished = false;
};

}  // namespace

struct wfa_server {
    wfa_ctx* ctx = nullptr;
    wfa_server_cfg cfg{};
    std::vector<std::unique_ptr<Engine>> engines;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> fifo;  // tickets with unadmitted pairs, arrival order
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    size_t reserved = 0, max_reserved = 0;
    uint64_t submitted = 0, completed = 0, batches = 0, pairs_done = 0;
    double busy_s = 0;
    std::chrono::steady_clock::time_point t0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

// Device bytes of one pair: staged sequences, packed words, descriptors and
// results, plus wavefront memory.  A pair with a fraction d of edits, a third
// each substitutions (cost x) and single-base gaps (cost o + e), scores
// about s = d * max(n, m) * (x + 2 (o + e)) / 3; its wavefronts hold about
// s^2 / (g e) offsets over all steps (12 bytes each with history), or one
// ring of (pre + 1) rows of n + m + 1 offsets (score only).  d = 6 %, the
// middle of the 1-10 % the server is sized for; a pair that needs more is
// still aligned exactly (the engine re-runs it with a larger arena slice).
size_t pair_bytes(const wfa_server_cfg& cfg, uint32_t n, uint32_t m) {
    const double x = cfg.pen.mismatch, o = cfg.pen.gap_open, e = cfg.pen.gap_extend;
    const double g = std::gcd(std::gcd(cfg.pen.mismatch, cfg.pen.gap_open), cfg.pen.gap_extend);
    const double L = std::max(n, m);
    size_t io = (size_t)n + m + 2 * (((size_t)n + 31) / 32 + ((size_t)m + 31) / 32) * 8 + 64;
    const double s = 0.06 * L * (x + 2 * (o + e)) / 3 + o + e;
    // a ring of full-width M/I/D rows of the score steps (all modes), and in
    // CIGAR mode the history: an offset and a 4-bit record per cell (about
    // s'^2 / e' cells) and a 16-byte table entry per step, plus the runs
    const double pre = std::max(x, o + e) / g;
    double wf = 12.0 * (pre + 2) * ((double)n + m + 3);
    if (cfg.mode == WFA_CIGAR) {
        const double cellb = m < 0xFFFF ? 2.5 : 4.5;  // 16-bit history offsets below 64 K
        wf += cellb * s * s / (g * e) + 16.0 * (s / g + 1);
        io += (size_t)(4.0 * 2 * (s / std::min(x, e) + 1));
    }
    return io + (size_t)wf;
}

// Run one merged batch on an engine (or the user's executor).
int run_batch(wfa_server* srv, Engine* eng, const wfa_request& rq, std::vector<int32_t>& scores,
              std::vector<uint32_t>& runs, std::vector<uint64_t>& offsets) {
    const bool cigar = srv->cfg.mode == WFA_CIGAR;
    const size_t n = rq.num_pairs;
    scores.assign(n, 0);
    offsets.assign(n + 1, 0);
    // runs: at most n + m + 1 per pair; a quarter of that covers any pair
    // within ~10 % divergence, and a larger need triggers one exact re-run
    size_t cap = 64;
    if (cigar)
        for (size_t i = 0; i < n; i++) cap += ((size_t)rq.pairs[i].p_len + rq.pairs[i].t_len) / 4 + 8;
    else
        cap = 0;
    for (int attempt = 0; attempt < 2; attempt++) {
        runs.assign(cap ? cap : 1, 0);
        size_t needed = 0;
        int rc;
        if (srv->cfg.executor) {
            rc = srv->cfg.executor(srv->cfg.executor_user, &rq, scores.data(),
                                   cigar ? runs.data() : nullptr, cap,
                                   cigar ? offsets.data() : nullptr, &needed);
        } else {
            BatchIO io{rq.patterns, rq.texts, rq.pairs, n, WFA_ASCII, WFA_HOST, srv->cfg.pen,
                       (wfa_mode)srv->cfg.mode, scores.data(), cigar ? runs.data() : nullptr, cap,
                       cigar ? offsets.data() : nullptr};
            int64_t bad = -1;
            rc = engine_align(eng, io, nullptr, &needed, &bad);
        }
        if (rc == WFA_E_CAPACITY && cigar && attempt == 0) {
            cap = needed;  // the next attempt holds every run
            continue;
        }
        if (rc == WFA_OK && cigar) runs.resize(needed);
        return rc;
    }
    return WFA_E_CAPACITY;
}

void worker_main(wfa_server* srv, Engine* eng) {
    if (eng) (void)hipSetDevice(eng->device);
    const bool cigar = srv->cfg.mode == WFA_CIGAR;
    const size_t max_chunk = (size_t)srv->cfg.max_chunk_pairs;
    for (;;) {
        std::vector<Piece> pieces;
        size_t est = 0;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            for (;;) {
                // form a batch from the head of the queue
                while (!srv->fifo.empty()) {
                    Request* r = srv->reqs[srv->fifo.front()].get();
                    size_t total = 0;
                    for (auto& p : pieces) total += p.count;
                    if (total >= max_chunk) break;
                    const size_t room = max_chunk - total;
                    size_t k = std::min(room, r->pairs.size() - r->next);
                    // shrink to the budget (a lone oversized pair still runs
                    // when nothing else holds memory, so nothing waits forever)
                    const size_t base = r->est_prefix[r->next];
                    while (k > 0 && srv->reserved + est + (r->est_prefix[r->next + k] - base) >
                                        srv->cfg.hbm_budget_bytes)
                        k = k / 2;
                    if (k == 0 && srv->reserved == 0 && est == 0 && pieces.empty()) k = 1;
                    if (k == 0) break;
                    pieces.push_back({r->ticket, r->next, k});
                    est += r->est_prefix[r->next + k] - base;
                    if (r->t_admit < 0) r->t_admit = srv->now();
                    r->next += k;
                    if (r->next == r->pairs.size()) srv->fifo.pop_front();
                    else break;  // budget or size limit reached inside this request
                }
                if (!pieces.empty()) break;
                if (srv->stop && srv->fifo.empty()) return;
                srv->cv_work.wait(lk);
            }
            srv->reserved += est;
            srv->max_reserved = std::max(srv->max_reserved, srv->reserved);
            srv->batches++;
        }
        // merged host batch.  A request's sequences never change after submit
        // and it cannot be released before this batch finishes, so only the
        // lookup needs the lock.
        std::vector<Request*> owners;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            for (auto& pc : pieces) owners.push_back(srv->reqs[pc.ticket].get());
        }
        std::vector<uint8_t> pat, txt;
        std::vector<wfa_pair> pairs;
        {
            for (size_t pi = 0; pi < pieces.size(); pi++) {
                const Piece& pc = pieces[pi];
                Request* r = owners[pi];
                for (size_t i = pc.first; i < pc.first + pc.count; i++) {
                    const wfa_pair& q = r->pairs[i];
                    wfa_pair d{pat.size(), txt.size(), q.p_len, q.t_len};
                    pat.insert(pat.end(), r->pat.begin() + q.p_start,
                               r->pat.begin() + q.p_start + q.p_len);
                    txt.insert(txt.end(), r->txt.begin() + q.t_start,
                               r->txt.begin() + q.t_start + q.t_len);
                    pairs.push_back(d);
                }
            }
        }
        pat.push_back(0);
        txt.push_back(0);
        wfa_request rq{pat.data(), txt.data(), pairs.data(), pairs.size()};
        std::vector<int32_t> scores;
        std::vector<uint32_t> runs;
        std::vector<uint64_t> offsets;
        const double t_run = srv->now();
        const int rc = run_batch(srv, eng, rq, scores, runs, offsets);
        if (rc != WFA_OK)
            std::fprintf(stderr, "libwfa server: batch of %zu pairs failed: %s\n", pairs.size(),
                         wfa_strerror(rc));
        const double t_end = srv->now();
        if (eng && std::getenv("WFA_DEBUG")) {
            const wfa_stats& L = eng->last;
            std::fprintf(stderr,
                         "libwfa server: batch %zu pairs, %.1f ms (engine: total %.1f, pack %.1f, "
                         "short %.1f, general %.1f, compact %.1f ms; short %llu, general %llu, "
                         "requeued %llu, chunks %d)\n",
                         pairs.size(), (t_end - t_run) * 1e3, L.ms_total, L.ms_pack, L.ms_align,
                         L.ms_general, L.ms_compact, (unsigned long long)L.short_pairs,
                         (unsigned long long)L.general_pairs, (unsigned long long)L.requeued,
                         L.host_chunks);
        }
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            srv->busy_s += t_end - t_run;
            srv->reserved -= est;
            srv->pairs_done += pairs.size();
            size_t at = 0;
            for (auto& pc : pieces) {
                Request* r = srv->reqs[pc.ticket].get();
                if (rc != WFA_OK) r->status = rc;
                for (size_t i = 0; i < pc.count; i++) r->scores[pc.first + i] = scores[at + i];
                if (cigar && rc == WFA_OK) {
                    std::vector<uint32_t> cnt(pc.count);
                    for (size_t i = 0; i < pc.count; i++)
                        cnt[i] = (uint32_t)(offsets[at + i + 1] - offsets[at + i]);
                    r->piece_runs[pc.first].assign(runs.begin() + offsets[at],
                                                   runs.begin() + offsets[at + pc.count]);
                    r->piece_counts[pc.first] = std::move(cnt);
                }
                at += pc.count;
                r->done_pairs += pc.count;
                if (r->done_pairs == r->pairs.size()) {
                    if (cigar) {
                        r->offsets.assign(r->pairs.size() + 1, 0);
                        size_t idx = 0;
                        for (auto& kv : r->piece_runs) {
                            const auto& cnt = r->piece_counts[kv.first];
                            r->runs.insert(r->runs.end(), kv.second.begin(), kv.second.end());
                            for (uint32_t c : cnt) {
                                r->offsets[idx + 1] = r->offsets[idx] + c;
                                idx++;
                            }
                        }
                        r->piece_runs.clear();
                        r->piece_counts.clear();
                    }
                    r->t_done = t_end;
                    r->finished = true;
                    srv->completed++;
                }
            }
        }
        srv->cv_done.notify_all();
        srv->cv_work.notify_all();
    }
}

}  // namespace

extern "C" int wfa_server_open(wfa_ctx* ctx, const wfa_server_cfg* cfg, wfa_server** out) {
    if (!out || !cfg) return WFA_E_INVAL;
    *out = nullptr;
    wfa::Pen pen;
    if (make_pen(cfg->pen, &pen) != WFA_OK) return WFA_E_INVAL;
    if (cfg->mode != WFA_SCORE && cfg->mode != WFA_CIGAR) return WFA_E_INVAL;
    if (!ctx && !cfg->executor) return WFA_E_INVAL;
    if (cfg->streams < 0 || cfg->streams > 64 || cfg->max_chunk_pairs < 0 || cfg->queue_limit < 0)
        return WFA_E_INVAL;
    auto* srv = new wfa_server();
    srv->ctx = ctx;
    srv->cfg = *cfg;
    if (!srv->cfg.hbm_budget_bytes) srv->cfg.hbm_budget_bytes = (size_t)64 << 30;
    if (!srv->cfg.streams) srv->cfg.streams = 4;
    if (!srv->cfg.max_chunk_pairs) srv->cfg.max_chunk_pairs = 65536;
    if (!srv->cfg.queue_limit) srv->cfg.queue_limit = 1 << 20;
    srv->t0 = std::chrono::steady_clock::now();
    const int S = srv->cfg.streams;
    for (int i = 0; i < S; i++) {
        if (cfg->executor) {
            srv->engines.emplace_back(nullptr);
            continue;
        }
        std::unique_ptr<Engine> e;
        {
            std::lock_guard<std::mutex> lk(ctx->idle_mu);
            if (!ctx->idle.empty()) {
                e = std::move(ctx->idle.back());
                ctx->idle.pop_back();
            }
        }
        if (e) {
            // an engine of a closed server: its buffers stay unless they
            // exceed this server's share of the budget
            e->ws.budget = srv->cfg.hbm_budget_bytes / S;
            if (e->ws.total > e->ws.budget) e->ws.release_all();
            e->last_valid = false;
        } else {
            e = std::make_unique<Engine>();
            const int rc = engine_init(e.get(), ctx->device, srv->cfg.hbm_budget_bytes / S);
            if (rc != WFA_OK) {
                engine_destroy(e.get());
                for (auto& x : srv->engines)
                    if (x) engine_destroy(x.get());
                delete srv;
                return rc;
            }
        }
        e->opt = ctx->opt;
        e->opt.use_graph = -1;  // batch sizes vary from launch to launch
        e->ends = ctx->ends;    // the context's free ends (global by default)
        e->heur = ctx->heur;    // and its heuristic (exact by default)
        srv->engines.push_back(std::move(e));
    }
    for (int i = 0; i < S; i++) srv->workers.emplace_back(worker_main, srv, srv->engines[i].get());
    *out = srv;
    return WFA_OK;
}

extern "C" size_t wfa_server_estimate_bytes(const wfa_server* srv, const wfa_request* req) {
    if (!srv || !req || (req->num_pairs && !req->pairs)) return 0;
    size_t b = 0;
    for (size_t i = 0; i < req->num_pairs; i++)
        b += pair_bytes(srv->cfg, req->pairs[i].p_len, req->pairs[i].t_len);
    return b;
}

extern "C" int wfa_server_submit(wfa_server* srv, const wfa_request* req, uint64_t* ticket) {
    if (!srv || !req || !ticket) return WFA_E_INVAL;
    if (req->num_pairs && (!req->pairs || !req->patterns || !req->texts)) return WFA_E_INVAL;
    auto r = std::make_unique<Request>();
    const size_t n = req->num_pairs;
    r->pairs.resize(n);
    r->est_prefix.assign(n + 1, 0);
    uint64_t pb = 0, tb = 0;
    for (size_t i = 0; i < n; i++) {
        const wfa_pair& q = req->pairs[i];
        if (q.p_len > WFA_MAX_LENGTH || q.t_len > WFA_MAX_LENGTH) return WFA_E_TOO_LONG;
        r->pairs[i] = {pb, tb, q.p_len, q.t_len};
        pb += q.p_len;
        tb += q.t_len;
        r->est_prefix[i + 1] = r->est_prefix[i] + pair_bytes(srv->cfg, q.p_len, q.t_len);
    }
    r->pat.resize(pb);
    r->txt.resize(tb);
    for (size_t i = 0; i < n; i++) {
        const wfa_pair& q = req->pairs[i];
        std::memcpy(r->pat.data() + r->pairs[i].p_start, req->patterns + q.p_start, q.p_len);
        std::memcpy(r->txt.data() + r->pairs[i].t_start, req->texts + q.t_start, q.t_len);
    }
    r->scores.assign(n, 0);
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        if (srv->stop) return WFA_E_INVAL;
        if (srv->fifo.size() >= (size_t)srv->cfg.queue_limit) return WFA_E_BUSY;
        r->ticket = srv->next_ticket++;
        r->t_submit = srv->now();
        *ticket = r->ticket;
        srv->submitted++;
        if (n == 0) {
            r->t_admit = r->t_done = r->t_submit;
            r->offsets.assign(1, 0);
            r->finished = true;
            srv->completed++;
        } else {
            srv->fifo.push_back(r->ticket);
        }
        srv->reqs[r->ticket] = std::move(r);
    }
    srv->cv_work.notify_all();
    srv->cv_done.notify_all();
    return WFA_OK;
}

extern "C" int wfa_server_poll(wfa_server* srv, uint64_t ticket, int64_t timeout_us,
                               wfa_result* out) {
    if (!srv || !out) return WFA_E_INVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto ready = [&]() {
        auto it = srv->reqs.find(ticket);
        return it == srv->reqs.end() || it->second->finished;
    };
    if (timeout_us < 0) {
        srv->cv_done.wait(lk, ready);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return WFA_E_BUSY;
    }
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return WFA_E_NOTFOUND;
    Request* r = it->second.get();
    out->num_pairs = r->pairs.size();
    out->scores = r->scores.data();
    out->cigar_runs = r->runs.data();
    out->cigar_offsets = srv->cfg.mode == WFA_CIGAR ? r->offsets.data() : nullptr;
    out->submit_time_s = r->t_submit;
    out->admit_time_s = r->t_admit;
    out->done_time_s = r->t_done;
    out->status = r->status;
    return WFA_OK;
}

extern "C" int wfa_server_release(wfa_server* srv, uint64_t ticket) {
    if (!srv) return WFA_E_INVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return WFA_E_NOTFOUND;
    if (!it->second->finished) return WFA_E_BUSY;
    srv->reqs.erase(it);
    return WFA_OK;
}

extern "C" int wfa_server_get_stats(const wfa_server* srv, wfa_server_stats* out) {
    if (!srv || !out) return WFA_E_INVAL;
    auto* s = const_cast<wfa_server*>(srv);
    std::unique_lock<std::mutex> lk(s->mu);
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->batches = s->batches;
    out->pairs = s->pairs_done;
    out->budget_bytes = s->cfg.hbm_budget_bytes;
    out->reserved_bytes = s->reserved;
    out->max_reserved_bytes = s->max_reserved;
    out->busy_s = s->busy_s;
    return WFA_OK;
}

extern "C" int wfa_server_close(wfa_server* srv) {
    if (!srv) return WFA_E_INVAL;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    for (auto& t : srv->workers) t.join();
    // engines go back to the context for the next server (up to 16 kept)
    for (auto& e : srv->engines) {
        if (!e) continue;
        if (e->stream) (void)hipStreamSynchronize(e->stream);
        std::lock_guard<std::mutex> lk(srv->ctx->idle_mu);
        if (srv->ctx->idle.size() < 16) {
            srv->ctx->idle.push_back(std::move(e));
        } else {
            engine_destroy(e.get());
        }
    }
    delete srv;
    return WFA_OK;
}
