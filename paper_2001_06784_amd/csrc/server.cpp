// Serving loop for clique-count requests (continuous batching).
//
// Requests arrive on any host thread.  Worker threads (each with its own
// context and HIP stream, so passes of different workers overlap on the
// GPU) take every pending request that fits the pass budget and count them
// in one pass over their disjoint union (pv_count_batch): requests that
// arrive while a pass runs are admitted by the next free worker.  Graphs
// stay resident on the device under their key (an LRU cache bounded in
// bytes); a request names its graph by key and brings the host CSR for the
// case that it is not resident.
//
// Device memory: the resident graphs are loaded through one loader context;
// idle graphs are evicted (least recently used first) beyond cache_bytes,
// and the loader's hard limit adds what the running passes may pin.  A pass admits requests while their
// estimated footprint (union copy, orientation, SCT workspace, per-vertex
// output rows) stays within batch_bytes; the worker context's hard limit is
// twice that plus 64 MiB for its tables.  A pass that still runs out of it
// is split in halves and retried, down to single requests, which then fail
// with PV_ENOMEM.
//
// Built on the public C ABI only (pivoter.h) plus HIP for the per-worker
// output buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pivoter.h"

namespace {

using Clock = std::chrono::steady_clock;

double us_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::micro>(b - a).count();
}

enum ReqState { PENDING = 0, RUNNING = 1, DONE = 2 };

struct Req {
    pv_request r{};
    Clock::time_point t_submit;
    ReqState state = PENDING;
    pv_result res{};
    size_t bytes = 0;  // admission footprint
};

struct CacheEntry {
    pv_graph *g = nullptr;
    size_t bytes = 0;
    int pins = 0;
    uint64_t last_use = 0;
};

// device bytes of a graph's CSR
// (row pointers, columns, and the handle's small block of device counters)
size_t csr_bytes(long long n, long long nnz) { return 4 * (size_t)(n + 1) + 4 * (size_t)std::max(nnz, 1ll) + 64; }

// HBM a request occupies during a pass: its share of the union copy and
// orientation (CSR twice, oriented CSR, peel key, order, degrees and
// frontiers), of the SCT workspace (the walk's first capacities: 2n + m/8
// work items of 32 bytes, double-buffered; n/2 universes of 64 rows, with
// member ids and visit totals for local counts; 4n prefix entries), and its
// per-vertex output rows
size_t pass_bytes(const pv_request &r, long long nnz) {
    const size_t n = (size_t)r.n, m = (size_t)nnz / 2;
    size_t b = 2 * csr_bytes((long long)n, nnz) + 4 * (n + 1) + 2 * (size_t)nnz + 32 * n;
    b += 2 * 32 * (2 * n + m / 8) + (n / 2) * 64 * 8 + 4 * 4 * n;
    if (r.kind == PV_REQ_VERTEX) {
        const size_t K = (size_t)(r.k_hi - r.k_lo + 1);
        b += (n / 2) * (64 * 4 + 8 + 2 * K * 16 + 16) + n * K * 16;
    }
    return b;
}

}  // namespace

struct pv_server {
    pv_server_cfg cfg{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Req> reqs;
    std::unordered_map<uint64_t, CacheEntry> cache;
    size_t cache_used = 0;
    uint64_t use_clock = 0;
    uint64_t next_ticket = 1;
    bool stopping = false;
    std::vector<std::thread> threads;
    std::vector<pv_ctx *> ctxs;
    std::vector<hipStream_t> streams;
    // resident graphs are loaded and freed through this context (budget
    // cache_bytes); a context is not thread-safe, so load_mu guards it
    std::mutex load_mu;
    pv_ctx *loader = nullptr;
    hipStream_t load_stream = nullptr;

    void worker(int w);
    // unpinned graphs to release, least recently used first, until the
    // resident bytes plus `extra` fit the cache (taken out of the cache
    // under mu; the caller frees them after unlocking)
    std::vector<pv_graph *> evict_locked(size_t extra);
    void free_graphs(const std::vector<pv_graph *> &gs);
    pv_status resident(const pv_request &r, pv_graph **out);
    void count_pass(pv_ctx *c, const std::vector<pv_graph *> &lg, const std::vector<pv_request> &rq,
                    int klo, int khi, uint64_t *d_local, std::vector<pv_u128> &counts,
                    std::vector<int32_t> &omega, std::vector<uint64_t> &ovf, std::vector<pv_status> &st,
                    std::vector<uint64_t> &lovf, int cap);
};

std::vector<pv_graph *> pv_server::evict_locked(size_t extra) {
    std::vector<pv_graph *> out;
    while (cache_used + extra > (size_t)cfg.cache_bytes) {
        auto victim = cache.end();
        for (auto it = cache.begin(); it != cache.end(); ++it)
            if (it->second.pins == 0 && (victim == cache.end() || it->second.last_use < victim->second.last_use))
                victim = it;
        if (victim == cache.end()) break;  // everything resident is in use
        cache_used -= victim->second.bytes;
        out.push_back(victim->second.g);
        cache.erase(victim);
    }
    return out;
}

void pv_server::free_graphs(const std::vector<pv_graph *> &gs) {
    if (gs.empty()) return;
    std::lock_guard<std::mutex> lk(load_mu);
    for (pv_graph *g : gs) (void)pv_graph_free(g);
}

// Make the request's graph resident (pinned once for the request).
pv_status pv_server::resident(const pv_request &r, pv_graph **out) {
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(r.graph_key);
        if (it != cache.end()) {
            it->second.pins++;
            it->second.last_use = ++use_clock;
            *out = it->second.g;
            return PV_OK;
        }
    }
    const size_t want = csr_bytes(r.n, r.row_ptr[r.n]);
    pv_graph *ng = nullptr;
    pv_status s = PV_ENOMEM;
    for (int attempt = 0; attempt < 2 && s == PV_ENOMEM; attempt++) {
        std::vector<pv_graph *> victims;
        {
            std::lock_guard<std::mutex> lk(mu);
            victims = evict_locked(want);
        }
        free_graphs(victims);
        std::lock_guard<std::mutex> lk(load_mu);
        s = pv_graph_load_csr(loader, r.n, r.row_ptr, r.col, 0, &ng);
    }
    if (s != PV_OK) return s;
    int32_t n = 0;
    int64_t m = 0;
    pv_graph_size(ng, &n, &m);
    pv_graph *dup = nullptr;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(r.graph_key);
        if (it != cache.end()) {  // another worker loaded it meanwhile
            dup = ng;
            it->second.pins++;
            it->second.last_use = ++use_clock;
            *out = it->second.g;
        } else {
            CacheEntry e;
            e.g = ng;
            e.bytes = csr_bytes(n, 2 * m);
            e.pins = 1;
            e.last_use = ++use_clock;
            cache.emplace(r.graph_key, e);
            cache_used += e.bytes;
            *out = ng;
        }
    }
    if (dup) free_graphs({dup});
    return PV_OK;
}

// One batched pass over lg (global counts for all k, per-vertex counts for
// klo..khi when khi > 0).  A pass that runs out of the worker's device
// budget is split in halves, down to single requests.
void pv_server::count_pass(pv_ctx *c, const std::vector<pv_graph *> &lg, const std::vector<pv_request> &rq,
                           int klo, int khi, uint64_t *d_local, std::vector<pv_u128> &counts,
                           std::vector<int32_t> &omega, std::vector<uint64_t> &ovf, std::vector<pv_status> &st,
                           std::vector<uint64_t> &lovf, int cap) {
    const int L = (int)lg.size();
    const int K = khi > 0 ? khi - klo + 1 : 0;
    const int cw = (cap + 63) / 64;
    std::vector<long long> voff(L + 1, 0);
    for (int j = 0; j < L; j++) voff[j + 1] = voff[j] + rq[j].n;
    std::vector<std::pair<int, int>> todo{{0, L}};
    while (!todo.empty()) {
        const int a = todo.back().first, b = todo.back().second;
        todo.pop_back();
        if (a >= b) continue;
        uint64_t lv = 0;
        std::vector<pv_status> sub((size_t)(b - a), PV_OK);
        pv_status pass = pv_count_batch(c, b - a, lg.data() + a, 0, counts.data() + (size_t)a * cap, cap,
                                        omega.data() + a, ovf.data() + (size_t)a * cw, K > 0 ? PV_VERTEX : PV_NONE,
                                        klo, khi, K > 0 ? (pv_u128 *)(d_local + (size_t)voff[a] * K * 2) : nullptr,
                                        &lv, sub.data(), nullptr);
        if (pass == PV_ENOMEM && b - a > 1) {
            const int mid = (a + b) / 2;
            todo.push_back({mid, b});
            todo.push_back({a, mid});
            continue;
        }
        for (int j = a; j < b; j++) {
            st[j] = (pass == PV_OK || pass == PV_EBUFSIZE || pass == PV_EOVERFLOW) ? sub[j - a] : pass;
            lovf[j] = lv;
        }
    }
}

void pv_server::worker(int w) {
    pv_ctx *c = ctxs[w];
    hipStream_t st = streams[w];
    (void)hipSetDevice(cfg.device);
    uint64_t *d_local = nullptr;
    size_t d_local_n = 0;  // u64 words
    uint64_t *h_local = nullptr;
    size_t h_local_n = 0;
    for (;;) {
        std::vector<uint64_t> batch;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stopping || !queue.empty(); });
            if (queue.empty()) break;  // stopping and nothing left
            // admit pending requests in arrival order while the pass budget
            // allows (the first one always: it was checked at submit)
            size_t used = 0;
            while (!queue.empty() && (int)batch.size() < cfg.max_batch) {
                Req &q = reqs[queue.front()];
                if (!batch.empty() && used + q.bytes > (size_t)cfg.batch_bytes) break;
                used += q.bytes;
                batch.push_back(queue.front());
                queue.pop_front();
                q.state = RUNNING;
            }
        }
        const Clock::time_point t0 = Clock::now();
        const int G = (int)batch.size();
        std::vector<pv_request> rs(G);
        {
            std::lock_guard<std::mutex> lk(mu);
            for (int i = 0; i < G; i++) rs[i] = reqs[batch[i]].r;
        }
        // make every graph resident; each request of the pass pins its
        // entry once
        std::vector<pv_graph *> gs(G, nullptr);
        std::vector<pv_status> sts(G, PV_OK);
        for (int i = 0; i < G; i++) sts[i] = resident(rs[i], &gs[i]);
        // one pass over the loaded graphs: global counts for all k, and
        // per-vertex counts over the union of the requested k ranges
        std::vector<int> live;
        int cap = 1, klo = 0, khi = 0;
        long long N = 0;
        std::vector<long long> voff(G, 0);
        for (int i = 0; i < G; i++) {
            if (sts[i] != PV_OK) continue;
            live.push_back(i);
            voff[i] = N;
            N += rs[i].n;
            cap = std::max(cap, rs[i].cap);
            if (rs[i].kind == PV_REQ_VERTEX) {
                klo = klo ? std::min(klo, rs[i].k_lo) : rs[i].k_lo;
                khi = std::max(khi, rs[i].k_hi);
            }
        }
        const int L = (int)live.size();
        const int K = klo ? khi - klo + 1 : 0;
        std::vector<pv_graph *> lg(L);
        std::vector<pv_request> lr(L);
        for (int j = 0; j < L; j++) {
            lg[j] = gs[live[j]];
            lr[j] = rs[live[j]];
        }
        std::vector<pv_u128> counts((size_t)std::max(L, 1) * cap);
        std::vector<int32_t> omega(std::max(L, 1));
        const int cw = (cap + 63) / 64;
        std::vector<uint64_t> ovf((size_t)std::max(L, 1) * cw);
        std::vector<pv_status> pst(std::max(L, 1), PV_OK);
        std::vector<uint64_t> plovf(std::max(L, 1), 0);
        pv_status pass = PV_OK;
        if (K > 0) {
            const size_t need = (size_t)std::max<long long>(N, 1) * K * 2;
            if (need > d_local_n) {
                if (d_local) (void)hipFree(d_local);
                d_local = nullptr;
                d_local_n = 0;
                if (hipMalloc((void **)&d_local, need * 8) == hipSuccess) {
                    d_local_n = need;
                } else {
                    (void)hipGetLastError();  // reported as PV_ENOMEM; no later launch check sees it
                    pass = PV_ENOMEM;
                }
            }
            if (pass == PV_OK && need > h_local_n) {
                if (h_local) (void)hipHostFree(h_local);
                h_local = nullptr;
                h_local_n = 0;
                if (hipHostMalloc((void **)&h_local, need * 8) == hipSuccess) {
                    h_local_n = need;
                } else {
                    (void)hipGetLastError();
                    pass = PV_ENOMEM;
                }
            }
        }
        if (pass == PV_OK && L > 0) {
            count_pass(c, lg, lr, klo, K > 0 ? khi : 0, d_local, counts, omega, ovf, pst, plovf, cap);
            if (K > 0 && N > 0) {
                if (hipMemcpyAsync(h_local, d_local, (size_t)N * K * 16, hipMemcpyDeviceToHost, st) != hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess)
                    pass = PV_EDEVICE;
            }
        }
        const Clock::time_point t1 = Clock::now();
        // hand the results to the requests' own buffers
        std::vector<pv_result> out(G);
        for (int j = 0; j < L; j++) {
            const int i = live[j];
            pv_result &r = out[i];
            r.status = pass;
            if (pass != PV_OK) continue;
            if (pst[j] != PV_OK && pst[j] != PV_EBUFSIZE && pst[j] != PV_EOVERFLOW) {
                r.status = pst[j];
                continue;
            }
            const uint64_t lovf = plovf[j];
            const pv_request &q = rs[i];
            r.omega = omega[j];
            const pv_u128 *row = counts.data() + (size_t)j * cap;
            for (int k = 0; k < q.cap; k++) q.counts[k] = row[k];
            bool any = false;
            for (int k = 0; k < cap; k++)
                if ((ovf[(size_t)j * cw + (k >> 6)] >> (k & 63)) & 1) {
                    any = true;
                    if (k < 64) r.overflow |= 1ull << k;
                }
            if (q.kind == PV_REQ_VERTEX) {
                const int Kq = q.k_hi - q.k_lo + 1;
                const int c0 = q.k_lo - klo;
                const uint64_t *src = h_local + (size_t)voff[i] * K * 2;
                for (long long v = 0; v < q.n; v++)
                    for (int kk = 0; kk < Kq; kk++) {
                        q.vertex_out[(size_t)v * Kq + kk].lo = src[((size_t)v * K + c0 + kk) * 2];
                        q.vertex_out[(size_t)v * Kq + kk].hi = src[((size_t)v * K + c0 + kk) * 2 + 1];
                    }
                r.local_overflow = lovf;
                if (lovf) any = true;
            }
            if (q.cap <= omega[j]) r.status = PV_EBUFSIZE;
            else if (any) r.status = PV_EOVERFLOW;
        }
        std::vector<pv_graph *> victims;
        {
        std::lock_guard<std::mutex> lk(mu);
        const Clock::time_point t2 = Clock::now();
        for (int i = 0; i < G; i++) {
            Req &q = reqs[batch[i]];
            q.res = out[i];
            q.res.total_us = us_between(q.t_submit, t2);
            if (sts[i] != PV_OK) q.res.status = sts[i];
            q.res.batch_size = G;
            q.res.queue_us = us_between(q.t_submit, t0);
            q.res.run_us = us_between(t0, t1);
            q.state = DONE;
            auto it = cache.find(rs[i].graph_key);
            if (sts[i] == PV_OK && it != cache.end() && it->second.pins > 0) it->second.pins--;
        }
        victims = evict_locked(0);
        cv_done.notify_all();
        }
        // released outside the server lock: a free waits for the loader's
        // stream, and submit / wait / the other workers need not wait for it
        free_graphs(victims);
    }
    if (d_local) (void)hipFree(d_local);
    if (h_local) (void)hipHostFree(h_local);
}

extern "C" pv_status pv_server_start(const pv_server_cfg *cfg, pv_server **out) {
    if (!cfg || !out || cfg->workers < 1 || cfg->max_batch < 1 || cfg->cache_bytes < 0 ||
        cfg->batch_bytes <= 0)
        return PV_EINVAL;
    *out = nullptr;
    pv_server *s = new (std::nothrow) pv_server();
    if (!s) return PV_ENOMEM;
    s->cfg = *cfg;
    if (hipSetDevice(cfg->device) != hipSuccess) {
        delete s;
        return PV_EINVAL;
    }
    if (hipStreamCreateWithFlags(&s->load_stream, hipStreamNonBlocking) != hipSuccess) {
        pv_server_stop(s);
        return PV_EDEVICE;
    }
    {
        pv_config lc{};
        lc.stream = s->load_stream;
        // the cache keeps at most cache_bytes of idle graphs; the graphs
        // pinned by running passes may pass that by what the passes admit
        lc.hbm_budget = cfg->cache_bytes + (int64_t)cfg->workers * cfg->batch_bytes;
        pv_status e = pv_init(cfg->device, &lc, &s->loader);
        if (e != PV_OK) {
            pv_server_stop(s);
            return e;
        }
    }
    for (int w = 0; w < cfg->workers; w++) {
        hipStream_t st = nullptr;
        // default priority: the passes of different workers overlap
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            pv_server_stop(s);
            return PV_EDEVICE;
        }
        s->streams.push_back(st);
        pv_config wc{};
        wc.stream = st;
        // the admission estimate is the soft bound; the hard limit leaves
        // room for estimates that fall short and for the context's own
        // tables (binomials, the peel's fixed-size buffers)
        wc.hbm_budget = 2 * cfg->batch_bytes + (64ll << 20);
        pv_ctx *c = nullptr;
        pv_status e = pv_init(cfg->device, &wc, &c);
        if (e != PV_OK) {
            pv_server_stop(s);
            return e;
        }
        s->ctxs.push_back(c);
    }
    for (int w = 0; w < cfg->workers; w++) s->threads.emplace_back([s, w] { s->worker(w); });
    *out = s;
    return PV_OK;
}

extern "C" pv_status pv_server_submit(pv_server *s, const pv_request *req, uint64_t *ticket) {
    if (!s || !req || !ticket || req->n < 0 || !req->row_ptr || !req->counts || req->cap < 1)
        return PV_EINVAL;
    if (req->kind != PV_REQ_GLOBAL && req->kind != PV_REQ_VERTEX) return PV_EINVAL;
    if (req->kind == PV_REQ_VERTEX &&
        (req->k_lo < 1 || req->k_hi < req->k_lo || req->k_hi - req->k_lo + 1 > 8 || !req->vertex_out))
        return PV_EINVAL;
    const long long nnz = req->row_ptr[req->n];
    if (nnz < 0 || (nnz > 0 && !req->col)) return PV_EINVAL;
    Req q;
    q.r = *req;
    q.t_submit = Clock::now();
    q.bytes = pass_bytes(*req, nnz);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return PV_ECANCELLED;
    // never admissible: larger than one pass may hold
    if (q.bytes > (size_t)s->cfg.batch_bytes) return PV_ENOMEM;
    const uint64_t t = s->next_ticket++;
    s->reqs.emplace(t, q);
    s->queue.push_back(t);
    *ticket = t;
    s->cv_work.notify_one();
    return PV_OK;
}

static pv_status take_result(pv_server *s, uint64_t ticket, pv_result *out) {
    auto it = s->reqs.find(ticket);
    if (it->second.state != DONE) return PV_EAGAIN;
    if (out) *out = it->second.res;
    s->reqs.erase(it);
    return PV_OK;
}

extern "C" pv_status pv_server_poll(pv_server *s, uint64_t ticket, pv_result *out) {
    if (!s) return PV_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->reqs.find(ticket) == s->reqs.end()) return PV_EINVAL;
    return take_result(s, ticket, out);
}

extern "C" pv_status pv_server_wait(pv_server *s, uint64_t ticket, int64_t timeout_us, pv_result *out) {
    if (!s) return PV_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->reqs.find(ticket) == s->reqs.end()) return PV_EINVAL;
    auto done = [&] { return s->reqs[ticket].state == DONE; };
    if (timeout_us < 0) s->cv_done.wait(lk, done);
    else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done)) return PV_EAGAIN;
    return take_result(s, ticket, out);
}

extern "C" pv_status pv_server_cancel(pv_server *s, uint64_t ticket) {
    if (!s) return PV_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return PV_EINVAL;
    if (it->second.state != PENDING) return PV_EAGAIN;  // already in a pass
    s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), ticket), s->queue.end());
    it->second.state = DONE;
    it->second.res = pv_result{};
    it->second.res.status = PV_ECANCELLED;
    s->cv_done.notify_all();
    return PV_OK;
}

extern "C" void pv_server_stop(pv_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        // requests not yet in a pass are cancelled
        for (uint64_t t : s->queue) {
            Req &q = s->reqs[t];
            q.state = DONE;
            q.res = pv_result{};
            q.res.status = PV_ECANCELLED;
        }
        s->queue.clear();
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
    for (auto &t : s->threads) t.join();
    for (auto &e : s->cache) (void)pv_graph_free(e.second.g);
    s->cache.clear();
    for (pv_ctx *c : s->ctxs) pv_fini(c);
    if (s->loader) pv_fini(s->loader);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    if (s->load_stream) (void)hipStreamDestroy(s->load_stream);
    delete s;
}

extern "C" pv_status pv_server_stats(pv_server *s, int32_t *resident, int64_t *resident_bytes,
                                     int32_t *pending) {
    if (!s) return PV_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (resident) *resident = (int32_t)s->cache.size();
    if (resident_bytes) *resident_bytes = (int64_t)s->cache_used;
    if (pending) *pending = (int32_t)s->queue.size();
    return PV_OK;
}
