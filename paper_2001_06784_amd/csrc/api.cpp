// Host runtime of libpivoter: contexts, graph handles, the orientation and
// SCT launch sequence, buffer management.  Implements include/pivoter.h.
//
// Launch sequence of one count (all on the context's stream):
//   orient:   cooperative peel -> out-degrees -> scan -> N+(v) -> root order
//   SCT:      leaves of empty roots; then level by level, the level kernel
//             takes the multi-word items, compact items and (level 0) the
//             roots, and emits the next level's items; the host reads the
//             emitted counts after each level.  If any work buffer filled up
//             the whole count is rerun with larger buffers (results are
//             never partially reused).
//   finalize: C_k = sum_{h,p} L[h][p] C(p, k-h) in exact u128.
#include "internal.h"
#include "pivoter.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <thread>
#include <memory>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

// ------------------------------------------------------------- errors

static thread_local char g_last_error[256] = "";

static void set_err(const char *what, hipError_t e) {
    snprintf(g_last_error, sizeof g_last_error, "%s: %s", what, hipGetErrorString(e));
    // the failed call is reported here; its error must not stay behind as
    // the thread's last error, where the next launch check would find it
    (void)hipGetLastError();
}

#define HIPCHK(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) {                        \
            set_err(#call, e_);                        \
            return (e_ == hipErrorOutOfMemory) ? PV_ENOMEM : PV_EDEVICE; \
        }                                              \
    } while (0)

#define PVCHK(call)                      \
    do {                                 \
        pv_status s_ = (call);           \
        if (s_ != PV_OK) return s_;      \
    } while (0)

// p must be device memory (or managed memory) of the context's device.
static pv_status require_device(int device, const void *p, const char *what) {
    hipPointerAttribute_t at;
    const hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) (void)hipGetLastError();
    if (e != hipSuccess || (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged) ||
        at.device != device) {
        snprintf(g_last_error, sizeof g_last_error, "%s must be device memory of device %d", what, device);
        return PV_EINVAL;
    }
    return PV_OK;
}

extern "C" const char *pv_strerror(pv_status s) {
    switch (s) {
        case PV_OK: return "ok";
        case PV_EINVAL: return "invalid argument";
        case PV_ENOTSIMPLE: return "graph is not a simple symmetric sorted CSR";
        case PV_ENOMEM: return "out of memory";
        case PV_EOVERFLOW: return "a count reached 2^128";
        case PV_EDEVICE: return "HIP device error";
        case PV_ETOOBIG: return "graph too large for this build";
        case PV_EBUFSIZE: return "output buffer too small";
        case PV_ECANCELLED: return "cancelled";
        case PV_EAGAIN: return "not admitted, retry";
        case PV_ETIMEDOUT: return "timed out";
        default: return "unknown status";
    }
}

extern "C" const char *pv_last_error(void) { return g_last_error; }

// waves per block of the level kernel
#define WAVES_PER_LAUNCH_BLOCK 4

// level-kernel variants: 0 global only; 1/2 per vertex, 8/16 k-slots, u128
// per-visit sums; 3 per edge; 4/5 per vertex, 8/16 k-slots, u64 sums
static void variant_params(int kv, int &kl, int &lk) {
    static const int KL[6] = {0, 8, 16, 8, 8, 16};
    static const int LK[6] = {PV_LK_VERTEX128, PV_LK_VERTEX128, PV_LK_VERTEX128, PV_LK_EDGE,
                              PV_LK_VERTEX64, PV_LK_VERTEX64};
    kl = KL[kv];
    lk = LK[kv];
}

static int variant_of(int kl, int lk) {
    if (kl == 0) return 0;
    if (lk == PV_LK_EDGE) return 3;
    if (lk == PV_LK_VERTEX64) return kl <= 8 ? 4 : 5;
    return kl <= 8 ? 1 : 2;
}

// ------------------------------------------------------------ handles

// Device bytes a context holds, against its configured limit.  Every
// device allocation of the library goes through DBuf::ensure, which charges
// the budget of the context whose entry point is running on this host
// thread (set by BudgetScope) and is refunded when the buffer is released.
struct Budget {
    std::atomic<long long> held{0};
    long long limit = 0;  // 0: no limit besides the device
};
static thread_local Budget *tl_budget = nullptr;

template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;  // elements
    Budget *charged = nullptr;
    size_t bytes = 0;
    void release() {
        if (p) (void)hipFree(p);
        if (charged) charged->held -= (long long)bytes;
        p = nullptr;
        n = 0;
        charged = nullptr;
        bytes = 0;
    }
    // ensure room for at least `need` elements (contents not kept)
    pv_status ensure(size_t need) {
        if (need <= n && p) return PV_OK;
        release();
        const size_t want = std::max<size_t>(need, 1) * sizeof(T);
        Budget *b = tl_budget;
        if (b && b->limit > 0 && b->held.load() + (long long)want > b->limit) {
            snprintf(g_last_error, sizeof g_last_error, "device memory budget of %lld bytes exceeded",
                     b->limit);
            return PV_ENOMEM;
        }
        hipError_t e = hipMalloc((void **)&p, want);
        if (e != hipSuccess) {
            set_err("hipMalloc", e);
            p = nullptr;
            // a failed allocation is reported here; clear the runtime's
            // last error so that a later launch check does not see it
            (void)hipGetLastError();
            return PV_ENOMEM;
        }
        n = std::max<size_t>(need, 1);
        bytes = want;
        charged = b;
        if (b) b->held += (long long)want;
        return PV_OK;
    }
};


// Scratch of one count call: the peel's temporaries and the SCT work
// buffers.  A context runs one call at a time, so all its graphs share one
// workspace (graph handles keep only the graph and its orientation).
struct Workspace {
    // peel / orientation temporaries
    DBuf<int> deg, fa, fb, scan, rcnt;  // rcnt: per-chunk out-degree histograms of the root order
    DBuf<int> owide;                    // orientation: the rows walked by a whole workgroup
    DBuf<int> lid, uverts, ldeg, lrp, lcol, bcnt, lrow;  // solo phase of the peel
    DBuf<PeelCtl> ctl;
    // SCT work buffers
    DBuf<CItem> citem[2];
    DBuf<uint64_t> mwitem[2];
    DBuf<uint64_t> hu_rows, u_rows;
    DBuf<int> hu_vl, u_gid, pref_pool;
    DBuf<int2> u_pref;
    DBuf<unsigned long long> hist, counters, phase, hsnap;
    DBuf<uint64_t> counts, ovf, vout_own;
    DBuf<int> omegas;
    DBuf<int> u_root;  // batches: root vertex of every universe
    // per-vertex prefix sums grouped by heavy root
    DBuf<int> u_grp, pg_cnt, pg_off, pg_pos, pg_list;
    // counts wider than u128: binomial table, per-k limbs, span and omega
    DBuf<uint64_t> wide_tab, wide_out;
    DBuf<int> wide_i;
    // frequency distributions of local counts
    DBuf<uint64_t> fq_keys, fq_vals;
    DBuf<int> fq_flags, fq_idx, fq_pos;
    // per-edge counts
    DBuf<int> ueid, weid;
    DBuf<uint64_t> umem, utot, escr;
    DBuf<uint64_t> epk, ewrap;  // packed pair charges and their carries (counts below 2^62)
    // persistent walk: the queues' slot flags and control block
    DBuf<int> cready, mready;
    DBuf<PersistCtl> pctl;
    // capacities: the walk's first ones follow the graph's size (see
    // run_sct_walk); a walk that fills a buffer runs again with the demand
    // it saw, and they stay for later calls.  Persistent walk: c_cap is
    // slots per slice of the compact queue, mw_cap slots of the multi-word
    // queue, each over the whole walk.
    static constexpr size_t C0 = 1 << 12, MW0 = 1 << 10, U0 = 1 << 10, PREF0 = 1 << 12;
    size_t c_cap = C0, mw_cap = MW0, u_cap = U0, pref_cap = PREF0;
    size_t pc_cap = C0, pm_cap = MW0;  // persistent walk: slots per compact slice, multi-word slots
    long long hu_budget = 1ll << 30;  // bytes of heavy universes per chunk

    // the walk's level buffers only (not the orientation's temporaries, the
    // tables, or outputs a caller's request points into)
    void release_level() {
        DBuf<int> *ib[] = {&hu_vl, &u_gid, &pref_pool, &u_root, &ueid, &weid, &u_grp, &pg_pos, &pg_list,
                           &cready, &mready};
        for (auto *b : ib) b->release();
        citem[0].release();
        citem[1].release();
        mwitem[0].release();
        mwitem[1].release();
        DBuf<uint64_t> *ub[] = {&hu_rows, &u_rows, &umem, &utot, &escr, &epk, &ewrap};
        for (auto *b : ub) b->release();
        u_pref.release();
        pctl.release();
    }

    void release() {
        DBuf<int> *ib[] = {&deg, &fa, &fb, &scan, &rcnt, &owide, &lid, &uverts, &ldeg, &lrp, &lcol,
                           &bcnt, &hu_vl, &u_gid, &pref_pool, &omegas, &u_root, &ueid, &weid,
                           &u_grp, &pg_cnt, &pg_off, &pg_pos, &pg_list, &wide_i, &fq_flags, &fq_idx,
                           &fq_pos, &lrow};
        for (auto *b : ib) b->release();
        ctl.release();
        citem[0].release();
        citem[1].release();
        mwitem[0].release();
        mwitem[1].release();
        DBuf<uint64_t> *ub[] = {&hu_rows, &u_rows, &counts, &ovf, &vout_own, &umem, &utot, &escr,
                                &epk, &ewrap, &wide_tab, &wide_out, &fq_keys, &fq_vals};
        for (auto *b : ub) b->release();
        u_pref.release();
        hist.release();
        counters.release();
        phase.release();
        hsnap.release();
        cready.release();
        mready.release();
        pctl.release();
        c_cap = C0;
        mw_cap = MW0;
        u_cap = U0;
        pref_cap = PREF0;
        pc_cap = C0;
        pm_cap = MW0;
    }
};

// Settings of the walk chosen by pv_autotune for one key.
struct TuneEntry {
    int dfs_max = 64, dfs_budget = 0, lane_max = PV_LANE_MAX;
    float ms_best = 0.f, ms_default = 0.f;
};

struct pv_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    Budget budget;
    std::string arch;                       // device part of the tuning keys
    std::string tune_path;                  // JSON cache file ("" : none)
    std::map<std::string, TuneEntry> tune;  // tuned settings by key
    DevInfo dev{};
    // exact binomials
    int bn = 0;
    int ts = 32;  // row stride of tab_pad (columns j = -16..ts-17)
    DBuf<uint64_t> tab, tab64, tab_pad;
    DBuf<uint8_t> bad;
    DBuf<int> fits64;
    int fits64_h[16] = {0};
    // launch arguments (device copy) and a pinned host staging copy
    DBuf<LevelArgs> d_args;
    LevelArgs *h_args = nullptr;
    int *h_io = nullptr;  // pinned readback slots
    PersistCtl *h_pctl = nullptr;  // pinned readback of the persistent walk's control block
    int level_blocks[6][4] = {};  // [kernel variant, see variant_of][unit kind, or PV_UNITS_ALL]
    bool persist = false;  // one persistent launch per walk (PV_PERSIST set) instead of level by level
    bool phase_on = false; // per-level phase times (PV_PHASE set; builds with PV_PHASE_TIMING)
    std::string record_path;  // PV_RECORD: a JSON line per count call appended here
    // cancellation and the watchdog: the device flag the walk's claims read,
    // set through its own stream while a call's kernels run
    int *d_abort = nullptr;
    // the stream that raises d_abort: created only for a context with a
    // watchdog or on its first pv_cancel (each stream takes one of the few
    // hardware queues, which the serving loop's workers share)
    hipStream_t abort_stream = nullptr;
    std::mutex abort_mu;
    std::atomic<int> cancel_req{0};
    bool timed_out = false;
    int timeout_ms = 0;
    int dfs_max = 64;
    int dfs_budget = 0;  // 0: chosen per request (see budget_of)
    int lane_max = PV_LANE_MAX;
    int prefix_rows = 0;  // PV_PREFIX_ROWS: N+(root) rows per LDS pass of the prefix sums (0: all that fit)
    // local counts (per vertex with 64-bit visit sums, per edge) added in
    // packed 32-bit halves when every count stays below 2^62 (PV_PACK=0
    // turns it off); pack_bias starts every half at that value instead of 0
    // (PV_PACK_BIAS, for tests: with a value near 2^32 the halves wrap after
    // a few additions)
    bool pack = true;
    uint32_t pack_bias = 0;
    bool debug = false;  // PV_DEBUG set: per-level buffer demands on stderr
    Workspace ws;
    // batches: the union graph (reused between calls) and its part table
    pv_graph *batch = nullptr;
    DBuf<BatchPart> parts;
    // device timing (HIP events on the context stream)
    bool timing = false;
    hipEvent_t ev[16] = {};
    // the unit kinds of one level run concurrently: kinds 1 and 2 on their
    // own streams (default priority), forked from and joined to the context
    // stream with events
    hipStream_t aux[2] = {nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_join[3] = {nullptr, nullptr, nullptr};
};

struct pv_graph {
    pv_ctx *ctx = nullptr;
    int n = 0;
    long long nnz = 0;
    DBuf<int> rp, col;
    int maxdeg = -1;  // largest degree (-1: not known); bounds the local counts
    // orientation
    bool oriented = false;
    int alpha = 0, subrounds = 0;
    int nheavy = 0, nnonzero = 0;
    DBuf<int> sub, odeg, orow, ocol, small, order;
    // batches (the union graph): graph of every vertex
    DBuf<int> vgraph;
    // per-edge counts: edge ids of the oriented CSR
    bool eids = false;
    DBuf<int> eup, o2e;
    pv_stats last{};
    std::atomic<int> busy{0};  // entry points running on this graph
    std::string deg_key;       // out-degree histogram part of the tuning key ("" : not yet)
};

static void tune_load(pv_ctx *c);

// A key's tuned settings on the context for the duration of one call.
struct TuneScope {
    pv_ctx *c;
    bool on = false;
    int dm = 0, db = 0, lm = 0;
    TuneScope(pv_ctx *c_, const std::string &key);
    ~TuneScope();
    TuneScope(const TuneScope &) = delete;
    TuneScope &operator=(const TuneScope &) = delete;
};
static pv_status tune_scope_for(pv_graph *g, int kind, int klo, int khi, int kmax,
                                std::unique_ptr<TuneScope> &scope);

// The context's budget for the allocations of one entry point.
struct BudgetScope {
    Budget *prev;
    explicit BudgetScope(pv_ctx *c) : prev(tl_budget) { tl_budget = c ? &c->budget : nullptr; }
    ~BudgetScope() { tl_budget = prev; }
};

// Graphs in use by an entry point (pv_graph_free refuses them meanwhile).
struct GraphUse {
    pv_graph *const *gs;
    int count;
    pv_graph *one;
    explicit GraphUse(pv_graph *g) : gs(&one), count(1), one(g) { mark(1); }
    GraphUse(pv_graph *const *list, int n) : gs(list), count(n), one(nullptr) { mark(1); }
    ~GraphUse() { mark(-1); }
    GraphUse(const GraphUse &) = delete;
    GraphUse &operator=(const GraphUse &) = delete;
    void mark(int d) {
        for (int i = 0; i < count; i++)
            if (gs[i]) gs[i]->busy += d;
    }
};

// small device scalars in g->small: alpha, three work cursors, emitted multi-word and
// compact item counts, flags, universes, prefix pool, omega, local overflow, error,
// root bounds
enum { SM_ALPHA = 0, SM_NEXT, SM_NEXT1, SM_NEXT2, SM_MWN, SM_CN, SM_FLAGS, SM_UN, SM_PREFN,
       SM_OMEGA, SM_LOVF, SM_ERR, SM_BOUNDS, SM_BOUNDS1, SM_COUNT };

extern "C" pv_status pv_init(int32_t device, const pv_config *cfg, pv_ctx **out) {
    if (!out) return PV_EINVAL;
    *out = nullptr;
    pv_config conf{};
    if (cfg) conf = *cfg;
    if (conf.hbm_budget < 0 || conf.dfs_max < 0 || conf.dfs_max > 64 || conf.lane_max < -1 || conf.timeout_ms < 0 ||
        conf.lane_max > PV_LANE_MAX || (conf.dfs_budget != 0 && (conf.dfs_budget < 16 || conf.dfs_budget > (1 << 20))))
        return PV_EINVAL;
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return PV_EINVAL;
    HIPCHK(hipSetDevice(device));
    pv_ctx *c = new (std::nothrow) pv_ctx();
    if (!c) return PV_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)conf.stream;
    c->budget.limit = conf.hbm_budget;
    BudgetScope scope(c);
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        set_err("hipGetDeviceProperties", e);
        delete c;
        return PV_EDEVICE;
    }
    // the allocation-free frequency entry point's scratch array on this
    // device (its address, resolved once per device with the device current)
    e = pv_freq_static_init(device);
    if (e != hipSuccess) {
        set_err("hipGetSymbolAddress", e);
        delete c;
        return PV_EDEVICE;
    }
    c->dev.device = device;
    c->dev.num_cu = prop.multiProcessorCount;
    {
        std::string an = prop.gcnArchName;
        c->arch = an.substr(0, an.find(':')) + "x" + std::to_string(prop.multiProcessorCount);
    }
    c->dev.lds_per_block = (int)prop.sharedMemPerBlock;
    c->dev.lds_per_cu = (int)prop.maxSharedMemoryPerMultiProcessor;
    if (hipHostMalloc((void **)&c->h_args, sizeof(LevelArgs)) != hipSuccess ||
        hipHostMalloc((void **)&c->h_io, 64 * sizeof(int)) != hipSuccess ||
        hipHostMalloc((void **)&c->h_pctl, sizeof(PersistCtl)) != hipSuccess) {
        delete c;
        return PV_ENOMEM;
    }
    if (c->d_args.ensure(1) != PV_OK) {
        delete c;
        return PV_ENOMEM;
    }
    for (int kv = 0; kv < 6; kv++)
        for (int mode = 0; mode < 4; mode++) {
            int kl, lk;
            variant_params(kv, kl, lk);
            int per_cu = pv_level_blocks_per_cu(kl, lk, mode);
            c->level_blocks[kv][mode] = std::max(1, per_cu) * c->dev.num_cu;
        }
    if (const char *env = getenv("PV_DFS_MAX")) c->dfs_max = std::max(1, std::min(64, atoi(env)));
    c->debug = getenv("PV_DEBUG") != nullptr;
    c->persist = getenv("PV_PERSIST") != nullptr;
    c->phase_on = getenv("PV_PHASE") != nullptr;
    if (const char *env = getenv("PV_RECORD")) c->record_path = env;
    if (const char *env = getenv("PV_DFS_BUDGET")) c->dfs_budget = std::max(16, std::min(1 << 20, atoi(env)));
    if (const char *env = getenv("PV_LANE_MAX")) c->lane_max = std::max(0, std::min(PV_LANE_MAX, atoi(env)));
    if (const char *env = getenv("PV_PREFIX_ROWS")) c->prefix_rows = std::max(0, atoi(env));
    if (const char *env = getenv("PV_PACK")) c->pack = atoi(env) != 0;
    if (const char *env = getenv("PV_PACK_BIAS")) c->pack_bias = (uint32_t)strtoul(env, nullptr, 0);
    if (const char *env = getenv("PV_HU_BUDGET")) {
        const long long b = atoll(env);
        if (b > 0) c->ws.hu_budget = b;
    }
    // the configuration's own settings come after the environment's
    if (conf.dfs_max > 0) c->dfs_max = conf.dfs_max;
    if (conf.dfs_budget > 0) c->dfs_budget = conf.dfs_budget;
    if (conf.lane_max > 0) c->lane_max = conf.lane_max;
    if (conf.lane_max < 0) c->lane_max = 0;
    if (c->budget.limit > 0) c->ws.hu_budget = std::min(c->ws.hu_budget, std::max(1ll << 20, c->budget.limit / 4));
    if (conf.tune_cache) {
        c->tune_path = conf.tune_cache;
        tune_load(c);
    }
    for (auto &ev : c->ev)
        if (hipEventCreate(&ev) != hipSuccess) {
            pv_fini(c);
            return PV_EDEVICE;
        }
    for (auto &st : c->aux)
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            pv_fini(c);
            return PV_EDEVICE;
        }
    if (hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess) {
        pv_fini(c);
        return PV_EDEVICE;
    }
    c->timeout_ms = conf.timeout_ms;
    if ((c->timeout_ms > 0 && hipStreamCreateWithFlags(&c->abort_stream, hipStreamNonBlocking) != hipSuccess) ||
        hipMalloc((void **)&c->d_abort, 256) != hipSuccess || hipMemset(c->d_abort, 0, 256) != hipSuccess) {
        (void)hipGetLastError();
        pv_fini(c);
        return PV_EDEVICE;
    }
    for (auto &ev : c->ev_join)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            pv_fini(c);
            return PV_EDEVICE;
        }
    *out = c;
    return PV_OK;
}

extern "C" void pv_fini(pv_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    // no work of this context may still be in flight when its memory goes
    (void)hipStreamSynchronize(c->stream);
    for (auto &st : c->aux)
        if (st) (void)hipStreamSynchronize(st);
    if (c->batch) pv_graph_free(c->batch);
    c->batch = nullptr;
    c->parts.release();
    c->ws.release();
    c->tab.release();
    c->tab64.release();
    c->tab_pad.release();
    c->bad.release();
    c->fits64.release();
    c->d_args.release();
    if (c->h_args) (void)hipHostFree(c->h_args);
    if (c->h_io) (void)hipHostFree(c->h_io);
    if (c->h_pctl) (void)hipHostFree(c->h_pctl);
    for (auto &st : c->aux)
        if (st) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    for (auto &ev : c->ev_join)
        if (ev) (void)hipEventDestroy(ev);
    for (auto &ev : c->ev)
        if (ev) (void)hipEventDestroy(ev);
    if (c->abort_stream) {
        (void)hipStreamSynchronize(c->abort_stream);
        (void)hipStreamDestroy(c->abort_stream);
    }
    if (c->d_abort) (void)hipFree(c->d_abort);
    delete c;
}

extern "C" pv_status pv_cancel(pv_ctx *c) {
    if (!c || !c->d_abort) return PV_EINVAL;
    std::lock_guard<std::mutex> lk(c->abort_mu);
    c->cancel_req.store(1);
    if (!c->abort_stream) {
        // on the context's device; the calling thread's current device is kept
        int prev = 0;
        HIPCHK(hipGetDevice(&prev));
        HIPCHK(hipSetDevice(c->device));
        const hipError_t e = hipStreamCreateWithFlags(&c->abort_stream, hipStreamNonBlocking);
        (void)hipSetDevice(prev);
        HIPCHK(e);
    }
    HIPCHK(hipMemsetAsync(c->d_abort, 1, sizeof(int), c->abort_stream));
    return PV_OK;
}

// Wait for the walk's work on stream s; with a timeout, poll and raise the
// abort flag once the call has run too long.  Then report a cancellation
// or a timeout of this call.
static pv_status wait_walk(pv_ctx *c, hipStream_t s, std::chrono::steady_clock::time_point t0) {
    if (c->timeout_ms <= 0) {
        HIPCHK(hipStreamSynchronize(s));
    } else {
        for (;;) {
            const hipError_t q = hipStreamQuery(s);
            if (q == hipSuccess) break;
            if (q != hipErrorNotReady) {
                set_err("hipStreamQuery", q);
                return PV_EDEVICE;
            }
            const double ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (!c->timed_out && ms > c->timeout_ms) {
                c->timed_out = true;
                HIPCHK(hipMemsetAsync(c->d_abort, 1, sizeof(int), c->abort_stream));
            }
            std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
    }
    if (c->timed_out) {
        snprintf(g_last_error, sizeof g_last_error, "call stopped after its %d ms timeout", c->timeout_ms);
        return PV_ETIMEDOUT;
    }
    if (c->cancel_req.load()) {
        snprintf(g_last_error, sizeof g_last_error, "call cancelled");
        return PV_ECANCELLED;
    }
    return PV_OK;
}

extern "C" pv_status pv_memory(const pv_ctx *c, int64_t *held_bytes) {
    if (!c || !held_bytes) return PV_EINVAL;
    *held_bytes = c->budget.held.load();
    return PV_OK;
}

// Peaks: each kernel runs `reps` times after one untimed run; the best
// rate counts.  The copy buffers are charged to the context's budget.
extern "C" pv_status pv_measure_peaks(pv_ctx *c, int64_t copy_bytes, pv_peaks *out) {
    if (!c || !out || copy_bytes < 0) return PV_EINVAL;
    BudgetScope bs(c);
    if (copy_bytes == 0) copy_bytes = (int64_t)1 << 30;
    copy_bytes = (copy_bytes + 4095) / 4096 * 4096;
    HIPCHK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    DBuf<uint8_t> a, b;
    DBuf<unsigned long long> sink;
    PVCHK(a.ensure((size_t)copy_bytes));
    PVCHK(b.ensure((size_t)copy_bytes));
    PVCHK(sink.ensure((size_t)PV_PEAK_BLOCKS * 256));
    HIPCHK(hipMemsetAsync(a.p, 0x5a, (size_t)copy_bytes, s));
    const int reps = 5, lds_iters = 1024, valu_iters = 256;
    hipEvent_t e0 = c->ev[14], e1 = c->ev[15];
    auto best_ms = [&](auto launch, float &ms_best) -> pv_status {
        ms_best = 0.f;
        HIPCHK(launch());
        for (int r = 0; r < reps; r++) {
            HIPCHK(hipEventRecord(e0, s));
            HIPCHK(launch());
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms_best == 0.f || ms < ms_best) ms_best = ms;
        }
        return PV_OK;
    };
    float ms_copy, ms_read, ms_lds, ms_valu;
    PVCHK(best_ms([&] { return pv_launch_peak_copy(a.p, b.p, copy_bytes, s); }, ms_copy));
    PVCHK(best_ms([&] { return pv_launch_peak_read(a.p, copy_bytes, (unsigned *)sink.p, s); }, ms_read));
    PVCHK(best_ms([&] { return pv_launch_peak_lds(lds_iters, 0, sink.p, s); }, ms_lds));
    PVCHK(best_ms([&] { return pv_launch_peak_valu(valu_iters, 0x1234567u, (unsigned *)sink.p, s); }, ms_valu));
    const double threads = (double)PV_PEAK_BLOCKS * 256.0;
    out->hbm_copy_gbs = 2.0 * (double)copy_bytes / (ms_copy * 1e-3) / 1e9;
    out->hbm_read_gbs = (double)copy_bytes / (ms_read * 1e-3) / 1e9;
    out->lds_read_gbs = threads * lds_iters * (double)PV_PEAK_LDS_READS * 8.0 / (ms_lds * 1e-3) / 1e9;
    out->valu_gops = threads * valu_iters * 8.0 * 8.0 * 2.0 / (ms_valu * 1e-3) / 1e9;
    out->ms_copy = ms_copy;
    out->ms_read = ms_read;
    out->ms_lds = ms_lds;
    out->ms_valu = ms_valu;
    return PV_OK;
}

extern "C" pv_status pv_set_stream(pv_ctx *c, void *stream) {
    if (!c) return PV_EINVAL;
    c->stream = (hipStream_t)stream;
    return PV_OK;
}

// Depth-first budget of a level: the set value, else 4096 with global
// counts alone and 8192 with local counts (each unit ends with a flush and
// a partial lane batch there, so fewer, larger units pay).  With local
// counts, a level whose units are fewer than 16 per wave lasts as long as
// its longest walk; 2048 then hands the rest of each long walk to the next
// level sooner.  Any budget gives the same tree and counts.
static int budget_of(const pv_ctx *c, bool local, long long units = -1, long long waves = 0) {
    if (c->dfs_budget > 0) return c->dfs_budget;
    if (!local) return 4096;
    if (units >= 0 && units < 16 * waves) return 2048;
    return 8192;
}

extern "C" pv_status pv_set_dfs_budget(pv_ctx *c, int32_t nodes) {
    if (!c || (nodes != 0 && (nodes < 16 || nodes > (1 << 20)))) return PV_EINVAL;
    c->dfs_budget = nodes;
    return PV_OK;
}

extern "C" pv_status pv_set_lane_max(pv_ctx *c, int32_t lane_max) {
    if (!c || lane_max < 0 || lane_max > PV_LANE_MAX) return PV_EINVAL;
    c->lane_max = lane_max;
    return PV_OK;
}

extern "C" pv_status pv_set_timing(pv_ctx *c, int32_t on) {
    if (!c) return PV_EINVAL;
    c->timing = on != 0;
    return PV_OK;
}

static float elapsed(pv_ctx *c, int a, int b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[a], c->ev[b]) != hipSuccess) return 0.f;
    return ms;
}

// tunable: largest |S| walked depth first (1..64)
extern "C" pv_status pv_set_dfs_max(pv_ctx *c, int32_t dfs_max) {
    if (!c || dfs_max < 1 || dfs_max > 64) return PV_EINVAL;
    c->dfs_max = dfs_max;
    return PV_OK;
}

// Binomials for a up to need - 1; the padded table's rows hold columns
// j = -16..ts-17 with ts >= ts_need
static pv_status ensure_binomials(pv_ctx *c, int need, int ts_need = 32) {
    if (need <= c->bn && ts_need <= c->ts) return PV_OK;
    int bn = std::max(need, c->bn);
    if (need > c->bn) bn = std::max(need, 2 * c->bn);
    const int ts = std::max(c->ts, (ts_need + 7) / 8 * 8);
    // the tables are rebuilt whole: until that succeeds the context has none
    // (a failed allocation below has released the old ones)
    c->bn = 0;
    c->ts = 0;
    PVCHK(c->tab.ensure((size_t)bn * bn * 2));
    PVCHK(c->bad.ensure((size_t)bn * bn));
    PVCHK(c->tab64.ensure((size_t)bn * 16));
    PVCHK(c->fits64.ensure(16));
    std::vector<int> ones(16, 1);
    HIPCHK(hipMemcpyAsync(c->fits64.p, ones.data(), 16 * sizeof(int), hipMemcpyHostToDevice, c->stream));
    PVCHK(c->tab_pad.ensure((size_t)2 * (bn + 1) * ts));
    HIPCHK(pv_launch_binomials(bn, c->tab.p, c->bad.p, c->tab64.p, c->fits64.p, c->stream));
    HIPCHK(pv_launch_binom_pad(bn, ts, c->tab.p, c->bad.p, c->tab_pad.p, c->stream));
    HIPCHK(hipMemcpyAsync(c->fits64_h, c->fits64.p, 16 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->bn = bn;
    c->ts = ts;
    return PV_OK;
}

// ------------------------------------------------------------- graphs

static pv_status graph_new(pv_ctx *c, int32_t n, long long nnz, pv_graph **out) {
    if (!c || !out || n < 0 || nnz < 0) return PV_EINVAL;
    if (nnz >= (1ll << 31) || n >= (1 << 30)) return PV_ETOOBIG;
    pv_graph *g = new (std::nothrow) pv_graph();
    if (!g) return PV_ENOMEM;
    g->ctx = c;
    g->n = n;
    g->nnz = nnz;
    pv_status s;
    if ((s = g->rp.ensure((size_t)n + 1)) != PV_OK || (s = g->col.ensure((size_t)nnz)) != PV_OK ||
        (s = g->small.ensure(SM_COUNT)) != PV_OK) {
        pv_graph_free(g);
        return s;
    }
    if (hipMemsetAsync(g->small.p, 0, SM_COUNT * sizeof(int), c->stream) != hipSuccess) {
        pv_graph_free(g);
        return PV_EDEVICE;
    }
    *out = g;
    return PV_OK;
}

static pv_status graph_validate(pv_graph *g, uint32_t flags) {
    pv_ctx *c = g->ctx;
    if (flags & PV_TRUST_INPUT) return PV_OK;
    // row pointers first: the row scan below must stay inside col[]
    HIPCHK(hipMemsetAsync(g->small.p + SM_ERR, 0, sizeof(int), c->stream));
    HIPCHK(pv_launch_check_rowptr(g->n, g->nnz, g->rp.p, g->small.p + SM_ERR, c->stream));
    int *err = c->h_io;
    HIPCHK(hipMemcpyAsync(err, g->small.p + SM_ERR, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (*err) return PV_ENOTSIMPLE;
    HIPCHK(pv_launch_validate(g->n, g->nnz, g->rp.p, g->col.p, g->small.p + SM_ERR, c->stream));
    HIPCHK(hipMemcpyAsync(err, g->small.p + SM_ERR, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return *err ? PV_ENOTSIMPLE : PV_OK;
}

// Repair of a host CSR (PV_DEDUP, PV_SYMMETRIZE): every row sorted, repeated
// entries and self loops dropped, and with PV_SYMMETRIZE the reverse of
// every entry added.  The row pointers must already be monotone and every
// column id in [0, n).
static pv_status repair_csr(int32_t n, const int32_t *rp, const int32_t *col, uint32_t flags,
                            std::vector<int32_t> &rp_out, std::vector<int32_t> &col_out) {
    const long long nnz = rp[n];
    for (long long i = 0; i < nnz; i++)
        if (col[i] < 0 || col[i] >= n) return PV_ENOTSIMPLE;
    std::vector<long long> deg((size_t)n + 1, 0);
    const bool sym = (flags & PV_SYMMETRIZE) != 0;
    for (int32_t v = 0; v < n; v++)
        for (int32_t i = rp[v]; i < rp[v + 1]; i++) {
            if (col[i] == v) continue;
            deg[v]++;
            if (sym) deg[col[i]]++;
        }
    std::vector<long long> off((size_t)n + 1, 0);
    for (int32_t v = 0; v < n; v++) off[v + 1] = off[v] + deg[v];
    if (off[n] >= (1ll << 31)) return PV_ETOOBIG;
    std::vector<int32_t> tmp((size_t)std::max<long long>(off[n], 1));
    std::vector<long long> fill(off.begin(), off.end() - 1);
    for (int32_t v = 0; v < n; v++)
        for (int32_t i = rp[v]; i < rp[v + 1]; i++) {
            const int32_t u = col[i];
            if (u == v) continue;
            tmp[fill[v]++] = u;
            if (sym) tmp[fill[u]++] = v;
        }
    rp_out.assign((size_t)n + 1, 0);
    col_out.clear();
    col_out.reserve((size_t)off[n]);
    for (int32_t v = 0; v < n; v++) {
        std::sort(tmp.begin() + off[v], tmp.begin() + off[v + 1]);
        const auto end = std::unique(tmp.begin() + off[v], tmp.begin() + off[v + 1]);
        col_out.insert(col_out.end(), tmp.begin() + off[v], end);
        rp_out[v + 1] = (int32_t)col_out.size();
    }
    return PV_OK;
}

extern "C" pv_status pv_graph_load_csr(pv_ctx *c, int32_t n, const int32_t *row_ptr,
                                       const int32_t *col, uint32_t flags, pv_graph **out) {
    if (!c || !out || n < 0 || !row_ptr || (n > 0 && row_ptr[n] > 0 && !col)) return PV_EINVAL;
    if (out) *out = nullptr;
    if (row_ptr[0] != 0 || row_ptr[n] < 0) return PV_ENOTSIMPLE;
    for (int32_t i = 0; i < n; i++)
        if (row_ptr[i + 1] < row_ptr[i]) return PV_ENOTSIMPLE;
    std::vector<int32_t> rrp, rcol;
    if (flags & (PV_DEDUP | PV_SYMMETRIZE)) {
        PVCHK(repair_csr(n, row_ptr, col, flags, rrp, rcol));
        row_ptr = rrp.data();
        col = rcol.data();
    }
    HIPCHK(hipSetDevice(c->device));
    BudgetScope scope(c);
    pv_graph *g = nullptr;
    PVCHK(graph_new(c, n, row_ptr[n], &g));
    hipError_t e = hipMemcpyAsync(g->rp.p, row_ptr, sizeof(int) * ((size_t)n + 1),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && g->nnz)
        e = hipMemcpyAsync(g->col.p, col, sizeof(int) * (size_t)g->nnz, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) {
        set_err("hipMemcpyAsync", e);
        pv_graph_free(g);
        return PV_EDEVICE;
    }
    pv_status s = graph_validate(g, flags);
    if (s != PV_OK) {
        pv_graph_free(g);
        return s;
    }
    int32_t dmax = 0;
    for (int32_t v = 0; v < n; v++) dmax = std::max(dmax, row_ptr[v + 1] - row_ptr[v]);
    g->maxdeg = dmax;
    *out = g;
    return PV_OK;
}

extern "C" pv_status pv_graph_load_csr_device(pv_ctx *c, int32_t n, int64_t nnz,
                                              const int32_t *d_row_ptr, const int32_t *d_col,
                                              uint32_t flags, pv_graph **out) {
    if (!c || !out || n < 0 || nnz < 0 || !d_row_ptr || (nnz > 0 && !d_col)) return PV_EINVAL;
    *out = nullptr;
    PVCHK(require_device(c->device, d_row_ptr, "d_row_ptr"));
    if (nnz > 0) PVCHK(require_device(c->device, d_col, "d_col"));
    HIPCHK(hipSetDevice(c->device));
    if (flags & (PV_DEDUP | PV_SYMMETRIZE)) {
        // repairs run on the host: a round trip of the CSR
        if (nnz >= (1ll << 31)) return PV_ETOOBIG;
        std::vector<int32_t> hrp((size_t)n + 1), hcol((size_t)std::max<long long>(nnz, 1));
        HIPCHK(hipMemcpyAsync(hrp.data(), d_row_ptr, sizeof(int) * hrp.size(), hipMemcpyDeviceToHost, c->stream));
        if (nnz)
            HIPCHK(hipMemcpyAsync(hcol.data(), d_col, sizeof(int) * (size_t)nnz, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (hrp[n] != nnz) return PV_EINVAL;
        return pv_graph_load_csr(c, n, hrp.data(), hcol.data(), flags, out);
    }
    BudgetScope scope(c);
    pv_graph *g = nullptr;
    PVCHK(graph_new(c, n, nnz, &g));
    hipError_t e = hipMemcpyAsync(g->rp.p, d_row_ptr, sizeof(int) * ((size_t)n + 1),
                                  hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && nnz)
        e = hipMemcpyAsync(g->col.p, d_col, sizeof(int) * (size_t)nnz, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) {
        set_err("hipMemcpyAsync", e);
        pv_graph_free(g);
        return PV_EDEVICE;
    }
    pv_status s = graph_validate(g, flags);
    if (s != PV_OK) {
        pv_graph_free(g);
        return s;
    }
    {
        // the largest degree, from a host copy of the row pointers
        std::vector<int32_t> hrp((size_t)n + 1);
        hipError_t e2 = hipMemcpyAsync(hrp.data(), g->rp.p, sizeof(int) * hrp.size(), hipMemcpyDeviceToHost, c->stream);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(c->stream);
        if (e2 != hipSuccess) {
            set_err("hipMemcpyAsync", e2);
            pv_graph_free(g);
            return PV_EDEVICE;
        }
        int32_t dmax = 0;
        for (int32_t v = 0; v < n; v++) dmax = std::max(dmax, hrp[v + 1] - hrp[v]);
        g->maxdeg = dmax;
    }
    *out = g;
    return PV_OK;
}

extern "C" pv_status pv_graph_free(pv_graph *g) {
    if (!g) return PV_OK;
    if (g->busy.load() > 0) {
        snprintf(g_last_error, sizeof g_last_error, "graph in use by a running count");
        return PV_EAGAIN;
    }
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    DBuf<int> *ib[] = {&g->rp, &g->col, &g->sub, &g->odeg, &g->orow, &g->ocol, &g->small, &g->order,
                       &g->vgraph, &g->eup, &g->o2e};
    for (auto *b : ib) b->release();
    delete g;
    return PV_OK;
}

extern "C" pv_status pv_graph_size(const pv_graph *g, int32_t *n, int64_t *m) {
    if (!g) return PV_EINVAL;
    if (n) *n = g->n;
    if (m) *m = g->nnz / 2;
    return PV_OK;
}

// --------------------------------------------------------- orientation

extern "C" pv_status pv_graph_orient(pv_graph *g, int32_t *alpha_out) {
    if (!g) return PV_EINVAL;
    pv_ctx *c = g->ctx;
    GraphUse use(g);
    BudgetScope scope(c);
    HIPCHK(hipSetDevice(c->device));
    const int n = g->n;
    PVCHK(g->sub.ensure(n));
    PVCHK(c->ws.deg.ensure(n));
    PVCHK(c->ws.fa.ensure(n));
    PVCHK(c->ws.fb.ensure(n));
    PVCHK(g->odeg.ensure(n));
    PVCHK(g->orow.ensure((size_t)n + 1));
    PVCHK(g->ocol.ensure((size_t)(g->nnz / 2)));
    PVCHK(c->ws.scan.ensure((size_t)n / 1024 + 2));
    PVCHK(c->ws.rcnt.ensure((size_t)pv_root_chunks(n) * (PV_MAX_ALPHA + 1)));
    PVCHK(g->order.ensure(n));
    PVCHK(c->ws.ctl.ensure(1));
    PVCHK(c->ws.lid.ensure(n));
    PVCHK(c->ws.uverts.ensure(PV_SOLO_MAX));
    PVCHK(c->ws.ldeg.ensure(PV_SOLO_MAX));
    PVCHK(c->ws.lrp.ensure(PV_SOLO_MAX + 1));
    PVCHK(c->ws.lcol.ensure((size_t)std::max<long long>(g->nnz, 1)));
    PVCHK(c->ws.bcnt.ensure(PV_PEEL_MAX_BLOCKS));
    PVCHK(c->ws.lrow.ensure(2 * PV_SOLO_MAX));
    PVCHK(c->ws.owide.ensure((size_t)(g->nnz / PV_ORIENT_BLOCK_ROW) + 2));
    hipStream_t s = c->stream;
    PeelCtl init;
    memset(&init, 0, sizeof init);
    init.minv[0] = init.minv[1] = 0x7fffffff;
    HIPCHK(hipMemcpyAsync(c->ws.ctl.p, &init, sizeof init, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(g->small.p + SM_ALPHA, 0, sizeof(int), s));
    HIPCHK(hipMemsetAsync(g->orow.p, 0, sizeof(int), s));
    if (n > 0) {
        if (c->timing) HIPCHK(hipEventRecord(c->ev[0], s));
        PeelArgs pa;
        pa.n = n;
        pa.rp = g->rp.p;
        pa.col = g->col.p;
        pa.deg = c->ws.deg.p;
        pa.sub = g->sub.p;
        pa.fa = c->ws.fa.p;
        pa.fb = c->ws.fb.p;
        pa.ctl = c->ws.ctl.p;
        pa.lid = c->ws.lid.p;
        pa.uverts = c->ws.uverts.p;
        pa.ldeg = c->ws.ldeg.p;
        pa.lrp = c->ws.lrp.p;
        pa.lcol = c->ws.lcol.p;
        pa.bcnt = c->ws.bcnt.p;
        pa.lrow = c->ws.lrow.p;
        HIPCHK(pv_launch_peel(c->dev, pa, s));
        if (c->timing) HIPCHK(hipEventRecord(c->ev[1], s));
        HIPCHK(pv_launch_orient(c->dev, n, g->rp.p, g->col.p, g->sub.p, g->odeg.p, g->orow.p,
                                g->ocol.p, g->small.p + SM_ALPHA, c->ws.scan.p, c->ws.lcol.p, c->ws.owide.p, s));
        HIPCHK(pv_launch_root_order(n, g->small.p + SM_ALPHA, g->odeg.p, c->ws.rcnt.p, pv_root_chunks(n),
                                    g->order.p, g->small.p + SM_BOUNDS, PV_LIGHT_MAX, s));
        if (c->timing) HIPCHK(hipEventRecord(c->ev[2], s));
    } else {
        HIPCHK(hipMemsetAsync(g->small.p + SM_BOUNDS, 0, 2 * sizeof(int), s));
    }
    int *io = c->h_io;
    HIPCHK(hipMemcpyAsync(io, g->small.p, SM_COUNT * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(io + 32, &c->ws.ctl.p->subrounds, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    g->alpha = io[SM_ALPHA];
    g->nheavy = io[SM_BOUNDS];
    g->nnonzero = io[SM_BOUNDS1];
    g->subrounds = io[32];
    if (n > 0 && io[34]) {
        snprintf(g_last_error, sizeof g_last_error, "peel grid barrier timed out");
        return PV_EDEVICE;
    }
    if (c->debug && n > 0) {
        PeelCtl pc;
        HIPCHK(hipMemcpy(&pc, c->ws.ctl.p, offsetof(PeelCtl, bar_flag), hipMemcpyDeviceToHost));
        const auto us = [&](int a, int b) { return (double)(pc.t_mark[b] - pc.t_mark[a]) * 0.01; };
        fprintf(stderr,
                "[pivoter] peel: %d sub-rounds, alpha %d; grid phase %.1f us (%d grid-wide sub-rounds, %d by "
                "one block, %d level changes); compaction of the last %d vertices %.1f us; solo phase %.1f us "
                "(%d sub-rounds)\n",
                pc.subrounds, pc.alpha, us(0, 1), pc.n_grid, pc.n_block, pc.n_levels, pc.n_solo, us(1, 2),
                us(2, 3), pc.subrounds - pc.n_grid - pc.n_block);
    }
    g->oriented = true;
    g->eids = false;
    if (c->timing && n > 0) {
        g->last.ms_peel = elapsed(c, 0, 1);
        g->last.ms_orient = elapsed(c, 1, 2);
    }
    if (alpha_out) *alpha_out = g->alpha;
    return PV_OK;
}

extern "C" pv_status pv_graph_export_order(pv_graph *g, int32_t *sub_host) {
    if (!g || (!sub_host && g->n > 0)) return PV_EINVAL;
    GraphUse use(g);
    if (!g->oriented) PVCHK(pv_graph_orient(g, nullptr));
    HIPCHK(hipSetDevice(g->ctx->device));
    if (g->n)
        HIPCHK(hipMemcpyAsync(sub_host, g->sub.p, sizeof(int) * (size_t)g->n, hipMemcpyDeviceToHost,
                              g->ctx->stream));
    HIPCHK(hipStreamSynchronize(g->ctx->stream));
    return PV_OK;
}

// ----------------------------------------------------------- the count

struct CountReq {
    int kmax = 0;
    int kl = 0;           // register k-slots for local counts (0: none)
    bool edge = false;    // local counts are per edge
    int lk = PV_LK_VERTEX128;  // level-kernel local kind (PV_LK_*)
    bool lane_ok = true;  // the lane tier may run (its per-vertex sums fit 64 bits)
    int graphs = 1;       // batch: parts of the disjoint union (one histogram each)
    const int *vgraph = nullptr;  // batch: part of every vertex
    int klo = 1, K = 0;
    bool wide_tab = false;     // some binomial the local sinks use passes 64 bits
    uint64_t *vout = nullptr;  // device [n][kstride] u128; this pass writes columns 0..K-1
    int kstride = 0;           // row stride of vout in slots (0: K)
    int c0 = 1;           // value of C_0
    // root subset (device order array + counts) or the whole graph
    const int *order = nullptr;
    int nheavy = 0, nlight = 0;
    bool whole = true;
    // a root subset's size (its roots and their out-degrees' sum), which
    // the first buffer capacities follow; -1: the graph's n and m
    long long size_n = -1, size_m = -1;
    const char *what = "count";  // the entry point, for run records
};

static pv_status run_sct_walk(pv_graph *g, const CountReq &rq);

// The walk; if it runs out of device memory (or of the context's budget)
// the SCT buffers are released, so the context stays usable for smaller
// work.
static pv_status run_sct(pv_graph *g, const CountReq &rq) {
    pv_status st = run_sct_walk(g, rq);
    if (st == PV_ENOMEM) g->ctx->ws.release();
    return st;
}

// The walk's level buffers at the workspace's capacities: the item queues,
// the universes and their per-count extras, the heavy roots' rows of one
// chunk.  PV_ENOMEM if they do not fit (the device or the budget).
static pv_status level_buffers(pv_ctx *c, pv_graph *g, const CountReq &rq, bool persist, int mw_stride, int chunk,
                               int W, int dpad) {
    const bool local = rq.kl > 0;
    (void)g;
    if (rq.vgraph) PVCHK(c->ws.u_root.ensure(c->ws.u_cap));
    if (persist) {
        PVCHK(c->ws.citem[0].ensure(c->ws.pc_cap * PV_QSLICES));
        PVCHK(c->ws.cready.ensure(c->ws.pc_cap * PV_QSLICES));
        PVCHK(c->ws.mwitem[0].ensure(c->ws.pm_cap * mw_stride));
        PVCHK(c->ws.mready.ensure(c->ws.pm_cap));
        PVCHK(c->ws.pctl.ensure(1));
    } else {
        for (int i = 0; i < 2; i++) {
            PVCHK(c->ws.citem[i].ensure(c->ws.c_cap));
            PVCHK(c->ws.mwitem[i].ensure(c->ws.mw_cap * mw_stride));
        }
    }
    PVCHK(c->ws.u_rows.ensure(c->ws.u_cap * 64));
    if (local) {
        PVCHK(c->ws.u_gid.ensure(c->ws.u_cap * 64));
        PVCHK(c->ws.u_pref.ensure(c->ws.u_cap));
        PVCHK(c->ws.pref_pool.ensure(c->ws.pref_cap));
    }
    if (local && !rq.edge) {
        PVCHK(c->ws.utot.ensure(c->ws.u_cap * 2 * rq.K * 2));
        PVCHK(c->ws.u_grp.ensure(c->ws.u_cap));
        PVCHK(c->ws.pg_pos.ensure(c->ws.u_cap));
        PVCHK(c->ws.pg_list.ensure(c->ws.u_cap));
        PVCHK(c->ws.pg_cnt.ensure((size_t)rq.nheavy + 1));
        PVCHK(c->ws.pg_off.ensure((size_t)rq.nheavy + 1));
        PVCHK(c->ws.scan.ensure((size_t)rq.nheavy / 1024 + 2));
    }
    if (rq.edge) {
        PVCHK(c->ws.umem.ensure(c->ws.u_cap * 64 * 2 * rq.K * 2));
        PVCHK(c->ws.utot.ensure(c->ws.u_cap * 3 * rq.K * 2));
        PVCHK(c->ws.ueid.ensure(c->ws.u_cap * 4096));
        const int wb = persist ? c->level_blocks[3][PV_UNITS_ALL] : c->level_blocks[3][PV_UNITS_LIGHT];
        PVCHK(c->ws.weid.ensure((size_t)wb * WAVES_PER_LAUNCH_BLOCK * 4096));
        // one region per wave; level by level, per unit kind too (the
        // kinds of a level run concurrently)
        const int eb = persist ? c->level_blocks[3][PV_UNITS_ALL]
                               : c->level_blocks[3][0] + c->level_blocks[3][1] + c->level_blocks[3][2];
        const size_t escr_words = (size_t)eb * WAVES_PER_LAUNCH_BLOCK * 2 * 64 * 2 * rq.K * 2;
        PVCHK(c->ws.escr.ensure(escr_words));
    }
    if (chunk > 0) {
        PVCHK(c->ws.hu_rows.ensure((size_t)chunk * W * dpad));
        PVCHK(c->ws.hu_vl.ensure((size_t)chunk * dpad));
    }
    // leave the device room for the launches themselves (scratch for the
    // kernels' spills, the runtime's own buffers): buffers that fill it to
    // the last gigabytes count as not fitting
    size_t free_b = 0, total_b = 0;
    HIPCHK(hipMemGetInfo(&free_b, &total_b));
    const size_t headroom = std::min<size_t>((size_t)4 << 30, total_b / 32);
    if (free_b < headroom) {
        snprintf(g_last_error, sizeof g_last_error, "level buffers leave %zu bytes of the device free", free_b);
        return PV_ENOMEM;
    }
    return PV_OK;
}

static pv_status run_sct_walk(pv_graph *g, const CountReq &rq) {
    pv_ctx *c = g->ctx;
    hipStream_t s = c->stream;
    // a new call: no cancellation or timeout of an earlier one applies
    const auto t_call = std::chrono::steady_clock::now();
    {
        std::lock_guard<std::mutex> lk(c->abort_mu);
        if (c->abort_stream) HIPCHK(hipStreamSynchronize(c->abort_stream));
        c->cancel_req.store(0);
    }
    c->timed_out = false;
    HIPCHK(hipMemsetAsync(c->d_abort, 0, sizeof(int), s));
    const int alpha = g->alpha;
    const int hd = alpha + 2;
    PVCHK(ensure_binomials(c, hd + 1));
    const int W = std::max(1, (alpha + 63) / 64);
    const int dpad = 64 * W;
    const int mw_stride = 3 * W + 1;
    const bool local = rq.kl > 0;
    int *io = c->h_io;
    // Local counts added in packed 32-bit halves (two values of k per 64-bit
    // atomic) when no count can reach 2^62.  A k-clique has a lowest vertex
    // r, and its other members lie in N+(r).  Through vertex v: r is v or a
    // neighbour of v, so c_k(v) <= (maxdeg + 1) * C(alpha, k - 1).  Through
    // edge uv: r is u, v or a common neighbour, so c_k(uv) <= n *
    // C(alpha, k - 2).  Per-vertex counts whose visit sums are 128 bits wide
    // are not packed.
    bool pack = false;
    const int kw = (rq.K + 1) / 2;
    // a row's words padded to a power of two (within one 64-byte line for
    // up to 8 words)
    int kws = 1;
    while (kws < kw) kws *= 2;
    const long long lrows_all = rq.edge ? g->nnz / 2 : (long long)g->n;
    if (local && c->pack && lrows_all > 0 && (rq.edge || rq.lk == PV_LK_VERTEX64) &&
        (rq.edge || g->maxdeg >= 0)) {
        const double mult = rq.edge ? (double)g->n : (double)g->maxdeg + 1.0;
        const int drop = rq.edge ? 2 : 1;  // C(alpha, k - drop)
        double worst = 0.0;
        for (int k = std::max(rq.klo, drop); k < rq.klo + rq.K; k++) {
            double b = 1.0;
            for (int i = 1; i <= k - drop && i <= alpha; i++) b = b * (double)(alpha - i + 1) / (double)i;
            if (k - drop > alpha) b = 0.0;
            worst = std::max(worst, mult * b);
        }
        pack = worst < 0x1p62;
    }

    // heavy roots per chunk, bounded by the universe budget
    const long long hu_bytes = (long long)W * dpad * 8 + (long long)dpad * 4;
    int chunk = (int)std::max<long long>(1, std::min<long long>(rq.nheavy, c->ws.hu_budget / hu_bytes));
    if (rq.nheavy == 0) chunk = 0;

    // first capacities from the graph's size (buffers only grow): most
    // calls then run the tree once; an overflow still reruns the whole walk
    // with the demand the counters saw
    {
        auto at_least = [](size_t &cap, long long want) {
            if ((long long)cap < want) cap = (size_t)want;
        };
        const long long n = rq.size_n >= 0 ? rq.size_n : g->n, m = rq.size_m >= 0 ? rq.size_m : g->nnz / 2;
        // (on a 1M-vertex, 9.9M-edge power-law graph: 0.52M items in the
        // fullest level, 187k multi-word items from 6.4k heavy roots, 251k
        // universes and 2.5M prefix entries over the whole walk)
        at_least(c->ws.c_cap, std::min<long long>(2 * n + m / 8, 1ll << 26));
        at_least(c->ws.u_cap, std::min<long long>(n / 2 + 1024, 1ll << 22));
        at_least(c->ws.pref_cap, std::min<long long>(4 * n + 4096, 1ll << 27));
        at_least(c->ws.mw_cap, std::min<long long>(rq.nheavy * 64ll + 1024, 1ll << 22));
        // the persistent walk's queues hold every item of the walk, not one
        // level's: twice the fullest level's demand, spread over the slices
        at_least(c->ws.pc_cap, std::min<long long>(2 * (2 * n + m / 8) / PV_QSLICES + 1024, 1ll << 26));
        at_least(c->ws.pm_cap, std::min<long long>(2 * rq.nheavy * 64ll + 1024, 1ll << 23));
    }
    const bool persist = c->persist;
    const int kli = variant_of(rq.kl, rq.lk);
    // the capacities the walk started from (a halved chunk never goes below)
    const size_t c_cap0 = c->ws.c_cap, mw_cap0 = c->ws.mw_cap;
    int resumes = 0;  // chunks run again after an overflow (global counts alone)
    for (int attempt = 0;; attempt++) {
        if (attempt > 48) return PV_ENOMEM;
        g->last.attempts = attempt + 1;
        // The level buffers hold one level's items of a chunk of heavy roots
        // (and of the light roots).  If they no longer fit the device or the
        // budget, the chunk is halved and the walk starts over: a level's
        // demand follows the heavy roots it descends from (R-MAT scale 18
        // truncated at k = 8 asks for 6.2e8 multi-word items in one level
        // with every heavy root in one chunk).
        pv_status lvl = level_buffers(c, g, rq, persist, mw_stride, chunk, W, dpad);
        if (lvl == PV_ENOMEM && chunk > 1) {
            c->ws.release_level();
            c->ws.c_cap = std::max(c_cap0, c->ws.c_cap / 2);
            c->ws.mw_cap = std::max(mw_cap0, c->ws.mw_cap / 2);
            chunk = (chunk + 1) / 2;
            if (c->debug)
                fprintf(stderr, "[pivoter] attempt %d: level buffers do not fit; %d heavy roots per chunk\n", attempt,
                        chunk);
            continue;
        }
        PVCHK(lvl);
        PVCHK(c->ws.hist.ensure((size_t)rq.graphs * hd * hd));
        PVCHK(c->ws.counters.ensure(PV_NCOUNTERS));
        if (rq.edge) HIPCHK(hipMemsetAsync(c->ws.escr.p, 0, c->ws.escr.n * 8, s));
        if (pack) {
            // the packed tables are an option: without room for them the
            // additions go straight to the output
            const size_t words = (size_t)lrows_all * kws;
            pv_status st = c->ws.epk.ensure(words);
            if (st == PV_OK) st = c->ws.ewrap.ensure(words);
            if (st == PV_ENOMEM) {
                c->ws.epk.release();
                c->ws.ewrap.release();
                pack = false;
            } else {
                PVCHK(st);
                HIPCHK(hipMemsetD32Async((hipDeviceptr_t)c->ws.epk.p, (int)c->pack_bias, 2 * words, s));
                HIPCHK(hipMemsetAsync(c->ws.ewrap.p, 0, words * 8, s));
            }
        }
        HIPCHK(hipMemsetAsync(c->ws.hist.p, 0, sizeof(unsigned long long) * (size_t)rq.graphs * hd * hd, s));
        HIPCHK(hipMemsetAsync(c->ws.counters.p, 0, PV_NCOUNTERS * sizeof(unsigned long long), s));
        // flags, u_n, pref_n, omega, lovf, and the checked build's failed line
        static_assert(SM_ERR == SM_FLAGS + 5, "walk scalars are contiguous");
        HIPCHK(hipMemsetAsync(g->small.p + SM_FLAGS, 0, 6 * sizeof(int), s));
        const size_t lrows = rq.edge ? (size_t)(g->nnz / 2) : (size_t)g->n;
        const int kstride = rq.kstride > 0 ? rq.kstride : rq.K;
        if (local && lrows) {
            if (kstride == rq.K) HIPCHK(hipMemsetAsync(rq.vout, 0, lrows * rq.K * 16, s));
            else HIPCHK(hipMemset2DAsync(rq.vout, (size_t)kstride * 16, 0, (size_t)rq.K * 16, lrows, s));
        }
        if (rq.whole)
            HIPCHK(pv_launch_sink_roots(g->n, g->order.p, g->small.p + SM_BOUNDS, c->ws.hist.p, hd,
                                        c->ws.counters.p, (local && !rq.edge) ? rq.vout : nullptr,
                                        rq.klo, kstride, rq.vgraph, s));

        bool overflow = false;
        bool io_fresh = false;  // io holds a readback of this attempt's flags
        int levels = 0;
        float ms_levels = 0.f;
        float ms_kind[3] = {0.f, 0.f, 0.f};
        uint32_t launches_kind[3] = {0, 0, 0};
        long long items = 0;
        // Chunks of heavy roots, the light roots with the first.  A walk of
        // global counts alone resumes at the chunk whose level overflowed:
        // the histogram and counters are restored to their state before it,
        // the buffers grow (or the chunk is halved until they fit), and only
        // that chunk runs again.  Universes live for one chunk then.  Local
        // counts accumulate into the caller's output and the universes'
        // owed totals, so they start the whole walk over instead.
        const bool resumable = !local && !persist;
        if (resumable) PVCHK(c->ws.hsnap.ensure((size_t)rq.graphs * hd * hd + PV_NCOUNTERS));
        int hbase = 0, nchunks = 0;
        for (bool done = false; !done && !overflow;) {
            const int hcount = (chunk > 0) ? std::min(chunk, rq.nheavy - hbase) : 0;
            const int ch = hbase == 0 ? 0 : 1;  // the light roots go with the first chunk
            if (resumable) {
                const size_t hw = (size_t)rq.graphs * hd * hd;
                HIPCHK(hipMemcpyAsync(c->ws.hsnap.p, c->ws.hist.p, hw * 8, hipMemcpyDeviceToDevice, s));
                HIPCHK(hipMemcpyAsync(c->ws.hsnap.p + hw, c->ws.counters.p, PV_NCOUNTERS * 8,
                                      hipMemcpyDeviceToDevice, s));
                HIPCHK(hipMemsetAsync(g->small.p + SM_UN, 0, sizeof(int), s));
            }
            int n_mw = 0, n_c = 0, cur = 0;
            // launch arguments shared by both forms of the walk
            auto fill_args = [&](LevelArgs &a, int level, int n_mw, int n_c, int cur, int nl) {
                memset(&a, 0, sizeof a);
                a.n = g->n;
                a.orow = g->orow.p;
                a.ocol = g->ocol.p;
                a.order = rq.order;
                a.heavy_base = hbase;
                a.nheavy = hcount;
                a.light_base = rq.nheavy;
                a.nlight = nl;
                a.kmax = rq.kmax;
                a.dfs_max = c->dfs_max;
                a.dfs_budget = budget_of(c, local);
                a.lane_max = (!local || rq.lane_ok) ? c->lane_max : 0;
                a.level = level;
                a.n_mw_in = n_mw;
                a.n_c_in = n_c;
                a.mw_in = c->ws.mwitem[cur].p;
                a.c_in = c->ws.citem[cur].p;
                a.mw_out = c->ws.mwitem[cur ^ 1].p;
                a.c_out = c->ws.citem[cur ^ 1].p;
                a.mw_out_n = g->small.p + SM_MWN;
                a.c_out_n = g->small.p + SM_CN;
                a.mw_cap = (int)c->ws.mw_cap;
                a.c_cap = (int)c->ws.c_cap;
                a.mw_stride = mw_stride;
                a.hu_rows = c->ws.hu_rows.p;
                a.hu_vl = c->ws.hu_vl.p;
                a.W = W;
                a.dpad = dpad;
                a.u_rows = c->ws.u_rows.p;
                a.u_gid = c->ws.u_gid.p;
                a.u_pref = c->ws.u_pref.p;
                a.u_n = g->small.p + SM_UN;
                a.u_cap = (int)c->ws.u_cap;
                a.pref_pool = c->ws.pref_pool.p;
                a.pref_n = g->small.p + SM_PREFN;
                a.pref_cap = (int)c->ws.pref_cap;
                a.u_grp = c->ws.u_grp.p;
                a.next = g->small.p + SM_NEXT;
                a.hist = c->ws.hist.p;
                a.hd = hd;
                a.counters = c->ws.counters.p;
                a.flags = g->small.p + SM_FLAGS;
                a.check = g->small.p + SM_ERR;
                a.vout = rq.vout;
                a.klo = rq.klo;
                a.K = rq.K;
                a.kstride = kstride;
                a.bin_pad = c->tab_pad.p;
                a.bin_pad_hi = rq.wide_tab ? c->tab_pad.p + (size_t)(c->bn + 1) * c->ts : nullptr;
                a.bin_bad = c->bad.p;
                a.bin_bn = c->bn;
                a.tab_stride = c->ts;
                a.lovf = g->small.p + SM_LOVF;
                a.sub = g->sub.p;
                a.o2e = rq.edge ? g->o2e.p : nullptr;
                a.umem = rq.edge ? c->ws.umem.p : nullptr;
                a.utot = local ? c->ws.utot.p : nullptr;
                a.ueid = rq.edge ? c->ws.ueid.p : nullptr;
                a.weid = rq.edge ? c->ws.weid.p : nullptr;
                a.escr = rq.edge ? c->ws.escr.p : nullptr;
                a.epk = pack ? c->ws.epk.p : nullptr;
                a.ewrap = pack ? c->ws.ewrap.p : nullptr;
                a.kw = kw;
                a.kws = kws;
                a.escr_wave0[0] = 0;
                a.escr_wave0[1] = c->level_blocks[3][0] * WAVES_PER_LAUNCH_BLOCK;
                a.escr_wave0[2] = (c->level_blocks[3][0] + c->level_blocks[3][1]) * WAVES_PER_LAUNCH_BLOCK;
                a.vgraph = rq.vgraph;
                a.u_root = rq.vgraph ? c->ws.u_root.p : nullptr;
                a.abort = c->d_abort;
            };
            if (persist) {
                // the whole walk of this chunk in one launch: every unit
                // from the device queues until the tree is done
                LevelArgs a;
                fill_args(a, 0, 0, 0, 0, (ch == 0) ? rq.nlight : 0);
                a.persist = 1;
                a.pctl = c->ws.pctl.p;
                a.cready = c->ws.cready.p;
                a.mready = c->ws.mready.p;
                a.c_scap = (int)c->ws.pc_cap;
                a.m_cap = (int)c->ws.pm_cap;
                a.c_out = c->ws.citem[0].p;
                a.mw_out = c->ws.mwitem[0].p;
                a.escr_wave0[0] = a.escr_wave0[1] = a.escr_wave0[2] = 0;
                const int blocks = c->level_blocks[kli][PV_UNITS_ALL];
                const long long waves = (long long)blocks * WAVES_PER_LAUNCH_BLOCK;
                // light roots: claimed in interleaved chunks, the last 8 per wave one at a time
                const long long nl = a.nlight;
                const long long lch = std::max(1ll, std::min(32ll, nl / (waves * 16)));
                const long long ln0 = (lch > 1) ? std::max(0ll, nl - 8 * waves) : 0;
                a.n0[PV_UNITS_LIGHT] = (int)ln0;
                a.nch[PV_UNITS_LIGHT] = (int)((ln0 + lch - 1) / lch);
                a.dfs_budget = budget_of(c, local);
                *c->h_args = a;
                HIPCHK(hipMemsetAsync(g->small.p + SM_NEXT, 0, 5 * sizeof(int), s));
                HIPCHK(hipMemsetAsync(c->ws.pctl.p, 0, sizeof(PersistCtl), s));
                HIPCHK(hipMemsetAsync(c->ws.cready.p, 0, c->ws.pc_cap * PV_QSLICES * sizeof(int), s));
                HIPCHK(hipMemsetAsync(c->ws.mready.p, 0, c->ws.pm_cap * sizeof(int), s));
                HIPCHK(hipMemcpyAsync(c->d_args.p, c->h_args, sizeof(LevelArgs), hipMemcpyHostToDevice, s));
                if (c->timing) HIPCHK(hipEventRecord(c->ev[3], s));
                HIPCHK(pv_launch_level(c->d_args.p, rq.kl, rq.lk, PV_UNITS_ALL, blocks, s));
                if (c->timing) HIPCHK(hipEventRecord(c->ev[4], s));
                HIPCHK(hipMemcpyAsync(io, g->small.p, SM_COUNT * sizeof(int), hipMemcpyDeviceToHost, s));
                PersistCtl *pcs = c->h_pctl;
                HIPCHK(hipMemcpyAsync(pcs, c->ws.pctl.p, sizeof(PersistCtl), hipMemcpyDeviceToHost, s));
                PVCHK(wait_walk(c, s, t_call));
                io_fresh = true;
                levels++;
                launches_kind[PV_UNITS_ITEMS]++;
                long long ctail_max = 0, pushed = (long long)(uint32_t)pcs->mtail.v;
                for (int sl = 0; sl < PV_QSLICES; sl++) {
                    ctail_max = std::max(ctail_max, (long long)(uint32_t)pcs->ctail[sl].v);
                    pushed += (long long)(uint32_t)pcs->ctail[sl].v;
                }
                if (c->timing) {
                    const float lv = elapsed(c, 3, 4);
                    ms_levels += lv;
                    ms_kind[PV_UNITS_ITEMS] += lv;
                }
                if (c->debug)
                    fprintf(stderr, "[pivoter] attempt %d chunk %d: persistent walk, %d blocks, items %lld "
                            "(largest slice %lld of %zu, multi-word %u of %zu), universes %d prefix %d, state %u\n",
                            attempt, ch, blocks, pushed, ctail_max, c->ws.pc_cap, (unsigned)(uint32_t)pcs->mtail.v,
                            c->ws.pm_cap, io[SM_UN], io[SM_PREFN], (unsigned)pcs->state.v);
                if (pcs->state.v & 3) {
                    snprintf(g_last_error, sizeof g_last_error, "persistent walk stopped: %s",
                             (pcs->state.v & 1) ? "no unit finished for 10 s" : "a queue slot was never written");
                    return PV_EDEVICE;
                }
                if (io[SM_FLAGS] & 1) {
                    overflow = true;
                    auto grow = [](size_t &cap, long long demand) {
                        if ((size_t)demand >= cap) cap = std::max(cap * 2, (size_t)(demand * 5 / 4) + 1024);
                    };
                    grow(c->ws.pc_cap, ctail_max);
                    grow(c->ws.pm_cap, (long long)(uint32_t)pcs->mtail.v);
                    grow(c->ws.u_cap, (unsigned)io[SM_UN]);
                    grow(c->ws.pref_cap, (unsigned)io[SM_PREFN]);
                    break;
                }
                items += pushed;
                nchunks++;
                hbase += hcount;
                done = hbase >= rq.nheavy;
                continue;
            }
            for (int level = 0;; level++) {
                LevelArgs a;
                fill_args(a, level, n_mw, n_c, cur, (ch == 0) ? rq.nlight : 0);
                const long long units = (long long)n_mw + n_c + (level == 0 ? (long long)a.nheavy + a.nlight : 0);
                if (units == 0) break;
                const int kli = variant_of(rq.kl, rq.lk);
                const long long mode_units[3] = {(long long)n_mw + (level == 0 ? a.nheavy : 0), n_c,
                                                 level == 0 ? a.nlight : 0};
                int mode_blocks[3];
                for (int mode = 0; mode < 3; mode++) {
                    const long long want = (mode_units[mode] + WAVES_PER_LAUNCH_BLOCK - 1) / WAVES_PER_LAUNCH_BLOCK;
                    mode_blocks[mode] = std::max(1, (int)std::min<long long>(c->level_blocks[kli][mode], want));
                    // claim chunks: about 16 claims per wave, at most 32 units
                    // each, interleaved over all but the last 8 units per
                    // wave; multi-word units are heavy, one at a time
                    const long long waves = (long long)mode_blocks[mode] * WAVES_PER_LAUNCH_BLOCK;
                    const long long chunk = (mode == PV_UNITS_MW)
                                                ? 1
                                                : std::max(1ll, std::min(32ll, mode_units[mode] / (waves * 16)));
                    const long long n0 = (chunk > 1) ? std::max(0ll, mode_units[mode] - 8 * waves) : 0;
                    a.n0[mode] = (int)n0;
                    a.nch[mode] = (int)((n0 + chunk - 1) / chunk);
                }
                a.dfs_budget = budget_of(c, local, units,
                                         (long long)c->level_blocks[kli][PV_UNITS_ITEMS] * WAVES_PER_LAUNCH_BLOCK);
                if (c->phase_on) {
                    // per-phase times of this level's units (libraries built
                    // with PV_PHASE_TIMING fill them)
                    PVCHK(c->ws.phase.ensure(48));
                    HIPCHK(hipMemsetAsync(c->ws.phase.p, 0, 48 * sizeof(unsigned long long), s));
                    a.phase = c->ws.phase.p;
                }
                *c->h_args = a;
                HIPCHK(hipMemsetAsync(g->small.p + SM_NEXT, 0, 5 * sizeof(int), s));
                HIPCHK(hipMemcpyAsync(c->d_args.p, c->h_args, sizeof(LevelArgs), hipMemcpyHostToDevice, s));
                if (c->timing) HIPCHK(hipEventRecord(c->ev[3], s));
                // the kinds of a level are independent (they only append to
                // the next level's queues): kinds 1 and 2 run on the
                // auxiliary streams, concurrently with kind 0
                HIPCHK(hipEventRecord(c->ev_fork, s));
                for (int mode = 0; mode < 3; mode++) {
                    if (mode_units[mode] == 0) continue;
                    hipStream_t ms = (mode == 0) ? s : c->aux[mode - 1];
                    if (ms != s) HIPCHK(hipStreamWaitEvent(ms, c->ev_fork, 0));
                    if (c->timing) HIPCHK(hipEventRecord(c->ev[8 + 2 * mode], ms));
                    HIPCHK(pv_launch_level(c->d_args.p, rq.kl, rq.lk, mode, mode_blocks[mode], ms));
                    if (c->timing) HIPCHK(hipEventRecord(c->ev[9 + 2 * mode], ms));
                    if (ms != s) {
                        HIPCHK(hipEventRecord(c->ev_join[mode], ms));
                        HIPCHK(hipStreamWaitEvent(s, c->ev_join[mode], 0));
                    }
                    launches_kind[mode]++;
                }
                if (c->timing) HIPCHK(hipEventRecord(c->ev[4], s));
                HIPCHK(hipMemcpyAsync(io, g->small.p, SM_COUNT * sizeof(int), hipMemcpyDeviceToHost, s));
                PVCHK(wait_walk(c, s, t_call));
                io_fresh = true;
                levels++;
                if (c->timing) {
                    const float lv = elapsed(c, 3, 4);
                    float km[3] = {0.f, 0.f, 0.f};
                    ms_levels += lv;
                    for (int mode = 0; mode < 3; mode++)
                        if (mode_units[mode]) ms_kind[mode] += (km[mode] = elapsed(c, 8 + 2 * mode, 9 + 2 * mode));
                    if (c->debug)
                        fprintf(stderr, "[pivoter] level %d: %.2f ms (multi-word %lld units %.2f ms, items %lld %.2f ms, "
                                "light roots %lld %.2f ms)\n", level, lv, mode_units[0], km[0], mode_units[1], km[1],
                                mode_units[2], km[2]);
                }
                if (c->phase_on) {
                    unsigned long long ph[48];
                    HIPCHK(hipMemcpy(ph, c->ws.phase.p, sizeof ph, hipMemcpyDeviceToHost));
                    for (int mode = 0; mode < 3; mode++) {
                        const unsigned long long *q = ph + 16 * mode;
                        if (!q[15]) continue;
                        fprintf(stderr, "[phase] level %d kind %d: waves %llu, per wave us: life %.1f", level, mode,
                                q[15], q[12] * 0.01 / q[15]);
                        for (int i = 0; i < 12; i++)
                            if (q[i]) fprintf(stderr, " p%d %.1f", i, q[i] * 0.01 / q[15]);
                        if (q[13])
                            fprintf(stderr, " | lane batches: %llu trips, %llu lane-nodes, use %.3f", q[13], q[14],
                                    (double)q[14] / (64.0 * (double)q[13]));
                        fprintf(stderr, "\n");
                    }
                }
                if (c->debug)
                    fprintf(stderr, "[pivoter] attempt %d level %d: mw %d items %d universes %d prefix %d "
                            "(caps %zu %zu %zu %zu)\n", attempt, level, io[SM_MWN], io[SM_CN], io[SM_UN],
                            io[SM_PREFN], c->ws.mw_cap, c->ws.c_cap, c->ws.u_cap, c->ws.pref_cap);
                if (io[SM_FLAGS] & 1) {
                    // a work buffer filled up: the counters kept counting every
                    // request, so they give the demand of this level; grow to it
                    overflow = true;
                    auto grow = [](size_t &cap, long long demand) {
                        if ((size_t)demand >= cap) cap = std::max(cap * 2, (size_t)(demand * 5 / 4) + 1024);
                    };
                    grow(c->ws.c_cap, (unsigned)io[SM_CN]);
                    grow(c->ws.mw_cap, (unsigned)io[SM_MWN]);
                    grow(c->ws.u_cap, (unsigned)io[SM_UN]);
                    grow(c->ws.pref_cap, (unsigned)io[SM_PREFN]);
                    break;
                }
                n_mw = io[SM_MWN];
                n_c = io[SM_CN];
                items += (long long)n_mw + n_c;
                cur ^= 1;
            }
            if (overflow && resumable) {
                // this chunk again, from the state before it
                const size_t hw = (size_t)rq.graphs * hd * hd;
                HIPCHK(hipMemcpyAsync(c->ws.hist.p, c->ws.hsnap.p, hw * 8, hipMemcpyDeviceToDevice, s));
                HIPCHK(hipMemcpyAsync(c->ws.counters.p, c->ws.hsnap.p + hw, PV_NCOUNTERS * 8,
                                      hipMemcpyDeviceToDevice, s));
                HIPCHK(hipMemsetAsync(g->small.p + SM_FLAGS, 0, sizeof(int), s));
                pv_status lv = level_buffers(c, g, rq, persist, mw_stride, chunk, W, dpad);
                while (lv == PV_ENOMEM && chunk > 1) {
                    c->ws.release_level();
                    c->ws.c_cap = std::max(c_cap0, c->ws.c_cap / 2);
                    c->ws.mw_cap = std::max(mw_cap0, c->ws.mw_cap / 2);
                    chunk = (chunk + 1) / 2;
                    if (c->debug)
                        fprintf(stderr, "[pivoter] level buffers do not fit; %d heavy roots per chunk\n", chunk);
                    lv = level_buffers(c, g, rq, persist, mw_stride, chunk, W, dpad);
                }
                PVCHK(lv);
                if (++resumes > 64) return PV_ENOMEM;
                overflow = false;
                continue;
            }
            if (overflow) break;
            nchunks++;
            hbase += hcount;
            done = hbase >= rq.nheavy;
        }
        g->last.heavy_chunks = nchunks;
        if (overflow) continue;
        if (local) {
            // what the universes' walks owe the vertices above them; the
            // device copy of the launch arguments still holds the last
            // level's (the universe buffers and outputs are the same for
            // every level)
            const int blocks = std::max(1, std::min(c->dev.num_cu * 16, (int)((io[SM_UN] + 3) / 4)));
            if (io_fresh) {  // no level ran: no universe, nothing to add
                if (rq.edge) {
                    HIPCHK(pv_launch_edge_prefix(c->d_args.p, blocks, s));
                } else {
                    const PrefixWork pw{c->ws.pg_cnt.p, c->ws.pg_off.p, c->ws.pg_pos.p, c->ws.pg_list.p,
                                        c->ws.scan.p};
                    const int rmax = PV_PREFIX_SLOTS / rq.K - 1;
                    const int rows = c->prefix_rows > 0 ? std::min(c->prefix_rows, rmax) : rmax;
                    HIPCHK(pv_launch_vertex_prefix(c->d_args.p, std::min(io[SM_UN], (int)c->ws.u_cap), rq.nheavy,
                                                   pw, rows, s));
                }
                if (pack)
                    HIPCHK(pv_launch_local_unpack(c->ws.epk.p, c->ws.ewrap.p, lrows_all, kw, kws, rq.K, rq.vout,
                                                  kstride, c->pack_bias, c->dev.num_cu, s));
                HIPCHK(hipMemcpyAsync(io, g->small.p, SM_COUNT * sizeof(int), hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
            }
        }
        if (io_fresh && (io[SM_FLAGS] & 4)) {
            snprintf(g_last_error, sizeof g_last_error, "edge id lookup failed");
            return PV_EDEVICE;
        }
        if (io_fresh && (io[SM_FLAGS] & 8)) {
            snprintf(g_last_error, sizeof g_last_error, "checked build: an invariant of the walk failed (sct.hip line %d)",
                     io[SM_ERR]);
            return PV_EDEVICE;
        }
        g->last.items = (uint64_t)items;
        g->last.kernel_kl = rq.kl;
        g->last.kernel_lk = rq.kl ? rq.lk : 0;
        g->last.truncated = rq.kmax > 0;
        g->last.levels = levels;
        g->last.ms_levels = ms_levels;
        for (int mode = 0; mode < 3; mode++) {
            g->last.ms_kind[mode] = ms_kind[mode];
            g->last.launches_kind[mode] = launches_kind[mode];
        }
        return PV_OK;
    }
}

// Read the walk's work counters into g->last.  The leaf sums come from the
// (h, p) leaf histogram; child work is one word per child (every node but
// the roots is a child) plus the multi-word children's extra words.
static pv_status read_counters(pv_graph *g, const CountReq &rq) {
    pv_ctx *c = g->ctx;
    hipStream_t s = c->stream;
    unsigned long long hcnt[PV_NCOUNTERS];
    HIPCHK(pv_launch_leaf_moments(c->ws.hist.p, g->alpha + 2, rq.graphs, c->ws.counters.p, s));
    HIPCHK(hipMemcpyAsync(hcnt, c->ws.counters.p, sizeof hcnt, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const unsigned long long roots = (unsigned long long)(rq.whole ? g->n : rq.size_n);
    g->last.nodes = hcnt[0];
    g->last.leaves = hcnt[1];
    g->last.work = hcnt[2];
    for (int mode = 0; mode < 3; mode++) g->last.work_kind[mode] = hcnt[4 + mode];
    g->last.child_work = hcnt[0] - std::min(hcnt[0], roots) + hcnt[PV_CTR_CHILD];
    g->last.leaf_hp = hcnt[PV_CTR_HP];
    g->last.leaf_pp = hcnt[PV_CTR_PP];
    return PV_OK;
}

// Run records: with PV_RECORD naming a file at pv_init, every count call
// appends one JSON line (the request, the graph, the walk's counters and
// device times, the status).
static std::mutex g_record_mu;

static void record_run(const pv_graph *g, const CountReq &rq, pv_status st) {
    const pv_ctx *c = g->ctx;
    if (c->record_path.empty()) return;
    const pv_stats &l = g->last;
    const char *local = rq.kl == 0 ? "none" : (rq.edge ? "edge" : "vertex");
    char line[1536];
    snprintf(line, sizeof line,
             "{\"t\": %.3f, \"call\": \"%s\", \"device\": \"%s\", \"n\": %d, \"m\": %lld, \"graphs\": %d, "
             "\"alpha\": %d, \"omega\": %d, \"k_max\": %d, \"local\": \"%s\", \"k_lo\": %d, \"k_hi\": %d, "
             "\"nodes\": %llu, \"leaves\": %llu, \"work\": %llu, \"child_work\": %llu, \"leaf_hp\": %llu, "
             "\"items\": %llu, \"attempts\": %d, \"heavy_chunks\": %d, \"levels\": %d, \"ms_peel\": %.3f, "
             "\"ms_orient\": %.3f, \"ms_levels\": %.3f, \"ms_finalize\": %.3f, \"status\": %d}\n",
             std::chrono::duration<double>(std::chrono::system_clock::now().time_since_epoch()).count(), rq.what,
             c->arch.c_str(), g->n, (long long)(g->nnz / 2), rq.graphs, l.alpha, l.omega, rq.kmax, local,
             rq.kl ? rq.klo : 0, rq.kl ? rq.klo + rq.K - 1 : 0, (unsigned long long)l.nodes,
             (unsigned long long)l.leaves, (unsigned long long)l.work, (unsigned long long)l.child_work,
             (unsigned long long)l.leaf_hp, (unsigned long long)l.items, l.attempts, l.heavy_chunks, l.levels,
             l.ms_peel, l.ms_orient, l.ms_levels, l.ms_finalize, (int)st);
    std::lock_guard<std::mutex> lk(g_record_mu);
    if (FILE *f = fopen(c->record_path.c_str(), "a")) {
        fputs(line, f);
        fclose(f);
    }
}

static pv_status finish_counts_body(pv_graph *g, const CountReq &rq, pv_u128 *counts, int32_t cap,
                                    int32_t *omega_out, uint64_t *overflow_bits, pv_stats *stats,
                                    uint64_t *local_ovf, pv_status *status);

static pv_status finish_counts(pv_graph *g, const CountReq &rq, pv_u128 *counts, int32_t cap,
                               int32_t *omega_out, uint64_t *overflow_bits, pv_stats *stats,
                               uint64_t *local_ovf, pv_status *status = nullptr) {
    const pv_status st = finish_counts_body(g, rq, counts, cap, omega_out, overflow_bits, stats, local_ovf, status);
    record_run(g, rq, st);
    return st;
}

static pv_status finish_counts_body(pv_graph *g, const CountReq &rq, pv_u128 *counts, int32_t cap,
                                    int32_t *omega_out, uint64_t *overflow_bits, pv_stats *stats,
                                    uint64_t *local_ovf, pv_status *status) {
    pv_ctx *c = g->ctx;
    hipStream_t s = c->stream;
    const int hd = g->alpha + 2;
    const int kcap = hd;
    const int nw = (kcap + 63) / 64;
    const int G = rq.graphs;  // 1, or the parts of a batch (one histogram each)
    PVCHK(c->ws.counts.ensure((size_t)G * kcap * 2));
    PVCHK(c->ws.ovf.ensure((size_t)G * nw));
    PVCHK(c->ws.omegas.ensure(G));
    HIPCHK(hipMemsetAsync(c->ws.ovf.p, 0, (size_t)G * nw * sizeof(uint64_t), s));
    HIPCHK(hipMemsetAsync(c->ws.omegas.p, 0, (size_t)G * sizeof(int), s));
    if (c->timing) HIPCHK(hipEventRecord(c->ev[5], s));
    HIPCHK(pv_launch_finalize(c->ws.hist.p, hd, c->tab.p, c->bad.p, c->bn, kcap, rq.kmax, rq.c0,
                              c->ws.counts.p, c->ws.ovf.p, c->ws.omegas.p, G, s));
    if (c->timing) HIPCHK(hipEventRecord(c->ev[6], s));
    std::vector<uint64_t> hc((size_t)G * kcap * 2), ho((size_t)G * nw);
    std::vector<int> hom(G);
    HIPCHK(hipMemcpyAsync(hc.data(), c->ws.counts.p, hc.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(ho.data(), c->ws.ovf.p, ho.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hom.data(), c->ws.omegas.p, (size_t)G * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(c->h_io, g->small.p, SM_COUNT * sizeof(int), hipMemcpyDeviceToHost, s));
    PVCHK(read_counters(g, rq));
    int omega_max = 0;
    for (int b = 0; b < G; b++) omega_max = std::max(omega_max, hom[b]);
    if (c->timing) g->last.ms_finalize = elapsed(c, 5, 6);
    g->last.alpha = g->alpha;
    g->last.omega = omega_max;
    g->last.subrounds = g->subrounds;
    if (stats) *stats = g->last;
    if (local_ovf) *local_ovf = c->h_io[SM_LOVF] ? ~0ull : 0ull;
    bool any_ovf = false, short_buf = false;
    const int cw = (cap + 63) / 64;
    for (int b = 0; b < G; b++) {
        const int omega = hom[b];
        if (omega_out) omega_out[b] = omega;
        const int top = (rq.kmax > 0) ? std::min(omega, rq.kmax) : omega;
        bool b_short = false, b_ovf = false;
        if (counts) {
            pv_u128 *row = counts + (size_t)b * cap;
            const uint64_t *src = hc.data() + (size_t)b * kcap * 2;
            for (int k = 0; k < cap; k++) {
                row[k].lo = (k < kcap) ? src[2 * k] : 0;
                row[k].hi = (k < kcap) ? src[2 * k + 1] : 0;
            }
            if (cap <= top) short_buf = b_short = true;
        }
        uint64_t *ob = overflow_bits ? overflow_bits + (size_t)b * cw : nullptr;
        if (ob) memset(ob, 0, sizeof(uint64_t) * (size_t)cw);
        for (int k = 0; k < kcap; k++) {
            if ((ho[(size_t)b * nw + (k >> 6)] >> (k & 63)) & 1) {
                any_ovf = b_ovf = true;
                if (ob && k < cap) ob[k >> 6] |= 1ull << (k & 63);
            }
        }
        if (status) status[b] = b_short ? PV_EBUFSIZE : (b_ovf ? PV_EOVERFLOW : PV_OK);
    }
    if (short_buf) return PV_EBUFSIZE;
    if (any_ovf || (local_ovf && *local_ovf)) return PV_EOVERFLOW;
    return PV_OK;
}

static pv_status prepare(pv_graph *g, bool reorient) {
    HIPCHK(hipSetDevice(g->ctx->device));
    g->last = pv_stats{};
    if (reorient || !g->oriented) {
        const pv_status st = pv_graph_orient(g, nullptr);
        if (st == PV_ENOMEM) g->ctx->ws.release();  // leave the context usable for smaller graphs
        if (st != PV_OK) return st;
    }
    if (g->alpha > PV_MAX_ALPHA) {
        snprintf(g_last_error, sizeof g_last_error, "degeneracy %d exceeds %d", g->alpha, PV_MAX_ALPHA);
        return PV_ETOOBIG;
    }
    return PV_OK;
}

static pv_status ensure_edge_ids(pv_graph *g) {
    if (g->eids) return PV_OK;
    pv_ctx *c = g->ctx;
    const long long m = g->nnz / 2;
    PVCHK(g->eup.ensure((size_t)g->n + 1));
    PVCHK(g->o2e.ensure((size_t)std::max<long long>(m, 1)));
    HIPCHK(hipMemsetAsync(g->eup.p, 0, sizeof(int), c->stream));
    HIPCHK(pv_launch_edge_ids(c->dev, g->n, g->rp.p, g->col.p, g->sub.p, g->orow.p, c->ws.fa.p,
                              g->eup.p, g->o2e.p, c->ws.scan.p, c->stream));
    g->eids = true;
    return PV_OK;
}

static pv_status setup_local(pv_graph *g, int kind, int klo, int khi, CountReq &rq) {
    if (kind == PV_NONE) return PV_OK;
    if (kind != PV_VERTEX && kind != PV_EDGE) return PV_EINVAL;
    // one pass keeps at most PV_MAX_LOCAL_K k-slots per lane
    if (klo < 1 || khi < klo || khi - klo + 1 > PV_MAX_LOCAL_K) return PV_EINVAL;
    // per-edge sums keep 8 k-slots per lane
    if (kind == PV_EDGE && khi - klo + 1 > 8) return PV_EINVAL;
    rq.klo = klo;
    rq.K = khi - klo + 1;
    rq.kl = rq.K <= 8 ? 8 : 16;
    rq.edge = kind == PV_EDGE;
    // the local paths use C(a, b), a <= alpha, b <= khi - 1; C(a, b) grows
    // with a, so the largest value used is at most max over b of C(alpha, b)
    // padded rows reach column klo + kl + 14 (a leaf's segment starts at
    // klo - h + 16 with h >= 1 and spans the kernel's kl slots)
    PVCHK(ensure_binomials(g->ctx, g->alpha + 3, klo + rq.kl + 15));
    unsigned __int128 cb = 1, cmax = 1;
    bool fits = true;  // all of them below 2^64
    for (int b = 1; b <= khi - 1 && b <= g->alpha && fits; b++) {
        cb = cb * (unsigned __int128)(g->alpha - b + 1) / (unsigned __int128)b;
        if (cb >> 64) fits = false;
        cmax = std::max(cmax, cb);
    }
    // per vertex: one 64-bit word per k-slot suffices when a universe
    // visit's sums stay below 2^64 (a visit walks at most dfs_budget nodes
    // plus two pivot chains, each leaf adding at most cmax)
    const unsigned __int128 visit_leaves = (unsigned __int128)budget_of(g->ctx, true) + 256;
    rq.lk = rq.edge ? PV_LK_EDGE
                    : ((fits && cmax * visit_leaves < ((unsigned __int128)1 << 64)) ? PV_LK_VERTEX64
                                                                                      : PV_LK_VERTEX128);
    // the lane tier (per vertex: 64-bit sums, 8 k-slots) adds up to one
    // batch of 64 subtrees of at most 34 nodes each (the largest SCT on 8
    // vertices) to a visit, and a lane's or a batch's sums stay below that
    rq.lane_ok = rq.lk == PV_LK_VERTEX64 && rq.kl == 8 &&
                 cmax * (visit_leaves + 64 * 34) < ((unsigned __int128)1 << 64);
    // binomials beyond 64 bits: the sinks add the table's high limbs too,
    // and flag the (exact) overflow of any count that needs one of 2^128 or
    // more (a leaf with at least 132 pivot vertices)
    rq.wide_tab = !fits;
    if (rq.edge) PVCHK(ensure_edge_ids(g));
    return PV_OK;
}

// pv_count on a prepared (oriented) graph with the context's settings
static pv_status count_body(pv_graph *g, int32_t k_max, pv_u128 *counts, int32_t cap, int32_t *omega_out,
                            uint64_t *overflow_bits, int32_t local_kind, int32_t k_lo, int32_t k_hi,
                            pv_u128 *local_out, uint64_t *local_ovf, pv_stats *stats) {
    CountReq rq;
    rq.kmax = k_max > 0 ? k_max : 0;
    PVCHK(setup_local(g, local_kind, k_lo, k_hi, rq));
    rq.vout = (uint64_t *)local_out;
    rq.order = g->order.p;
    rq.nheavy = g->nheavy;
    rq.nlight = g->nnonzero - g->nheavy;
    PVCHK(run_sct(g, rq));
    return finish_counts(g, rq, counts, cap, omega_out, overflow_bits, stats, local_ovf);
}

// pv_count without the tuning cache (pv_autotune times settings with it)
static pv_status count_untuned(pv_graph *g, int32_t reorient, int32_t k_max, pv_u128 *counts, int32_t cap,
                               int32_t *omega_out, uint64_t *overflow_bits, int32_t local_kind, int32_t k_lo,
                               int32_t k_hi, pv_u128 *local_out, uint64_t *local_ovf, pv_stats *stats) {
    if (!g || cap < 0 || (cap > 0 && !counts)) return PV_EINVAL;
    if (local_kind != PV_NONE && !local_out) return PV_EINVAL;
    if (local_kind != PV_NONE) PVCHK(require_device(g->ctx->device, local_out, "local_out"));
    GraphUse use(g);
    BudgetScope scope(g->ctx);
    PVCHK(prepare(g, reorient != 0));
    return count_body(g, k_max, counts, cap, omega_out, overflow_bits, local_kind, k_lo, k_hi, local_out,
                      local_ovf, stats);
}

extern "C" pv_status pv_count(pv_graph *g, int32_t reorient, int32_t k_max, pv_u128 *counts,
                              int32_t cap, int32_t *omega_out, uint64_t *overflow_bits,
                              int32_t local_kind, int32_t k_lo, int32_t k_hi, pv_u128 *local_out,
                              uint64_t *local_ovf, pv_stats *stats) {
    if (!g || cap < 0 || (cap > 0 && !counts)) return PV_EINVAL;
    if (local_kind != PV_NONE && !local_out) return PV_EINVAL;
    if (local_kind != PV_NONE) PVCHK(require_device(g->ctx->device, local_out, "local_out"));
    GraphUse use(g);
    BudgetScope scope(g->ctx);
    PVCHK(prepare(g, reorient != 0));
    std::unique_ptr<TuneScope> tuned;
    PVCHK(tune_scope_for(g, local_kind, k_lo, k_hi, k_max, tuned));
    return count_body(g, k_max, counts, cap, omega_out, overflow_bits, local_kind, k_lo, k_hi, local_out,
                      local_ovf, stats);
}

extern "C" pv_status pv_count_global(pv_graph *g, int32_t k_max, pv_u128 *counts, int32_t cap,
                                     int32_t *omega_out, uint64_t *overflow_bits, pv_stats *stats) {
    return pv_count(g, 0, k_max, counts, cap, omega_out, overflow_bits, PV_NONE, 0, 0, nullptr,
                    nullptr, stats);
}

extern "C" pv_status pv_count_global_wide(pv_graph *g, int32_t k_max, uint64_t *counts, int32_t cap,
                                          int32_t limbs, int32_t *omega_out, uint64_t *overflow_bits,
                                          pv_stats *stats) {
    if (!g || cap < 0 || (cap > 0 && !counts) || limbs < 1) return PV_EINVAL;
    pv_ctx *c = g->ctx;
    GraphUse use(g);
    BudgetScope scope(c);
    PVCHK(prepare(g, false));
    CountReq rq;
    rq.kmax = k_max > 0 ? k_max : 0;
    rq.what = "wide";
    PVCHK(setup_local(g, PV_NONE, 0, 0, rq));
    rq.order = g->order.p;
    rq.nheavy = g->nheavy;
    rq.nlight = g->nnonzero - g->nheavy;
    PVCHK(run_sct(g, rq));
    hipStream_t s = c->stream;
    const int hd = g->alpha + 2;
    // the binomials needed reach p <= the largest h + p of a leaf
    PVCHK(c->ws.wide_i.ensure(2));
    HIPCHK(hipMemsetAsync(c->ws.wide_i.p, 0, 2 * sizeof(int), s));
    if (c->timing) HIPCHK(hipEventRecord(c->ev[5], s));
    HIPCHK(pv_launch_count_wide(c->ws.hist.p, hd, 0, 0, 0, c->ws.wide_i.p, nullptr, 0, 0, 0, nullptr, nullptr, 0,
                                s));
    int span = 0;
    HIPCHK(hipMemcpyAsync(&span, c->ws.wide_i.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int bn = span + 1;
    const int tl = (bn + 63) / 64;  // C(p, j) < 2^p
    const int W = tl + 1;           // any count: histogram total < 2^64
    const int kcap = bn;
    const size_t tab_words = (size_t)bn * bn * tl;
    if (tab_words * 8 > ((size_t)2 << 30)) {
        snprintf(g_last_error, sizeof g_last_error, "binomial table for clique number %d exceeds 2 GiB", span);
        return PV_ENOMEM;
    }
    PVCHK(c->ws.wide_tab.ensure(tab_words));
    PVCHK(c->ws.wide_out.ensure((size_t)kcap * W));
    HIPCHK(pv_launch_count_wide(c->ws.hist.p, hd, kcap, rq.kmax, rq.c0, nullptr, c->ws.wide_tab.p, bn, tl, W,
                                c->ws.wide_out.p, c->ws.wide_i.p + 1, 1, s));
    if (c->timing) HIPCHK(hipEventRecord(c->ev[6], s));
    std::vector<uint64_t> hc((size_t)kcap * W);
    int omega = 0;
    HIPCHK(hipMemcpyAsync(hc.data(), c->ws.wide_out.p, hc.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&omega, c->ws.wide_i.p + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    PVCHK(read_counters(g, rq));
    if (c->timing) g->last.ms_finalize = elapsed(c, 5, 6);
    g->last.alpha = g->alpha;
    g->last.omega = omega;
    g->last.subrounds = g->subrounds;
    if (stats) *stats = g->last;
    if (omega_out) *omega_out = omega;
    const int cw = (cap + 63) / 64;
    if (overflow_bits) memset(overflow_bits, 0, sizeof(uint64_t) * (size_t)cw);
    bool any_ovf = false;
    for (int k = 0; k < cap; k++) {
        uint64_t *row = counts + (size_t)k * limbs;
        for (int l = 0; l < limbs; l++) row[l] = (k < kcap && l < W) ? hc[(size_t)k * W + l] : 0ull;
        bool ovf = false;
        for (int l = limbs; k < kcap && l < W; l++) ovf = ovf || hc[(size_t)k * W + l] != 0;
        if (ovf) {
            any_ovf = true;
            if (overflow_bits) overflow_bits[k >> 6] |= 1ull << (k & 63);
        }
    }
    const int top = (rq.kmax > 0) ? std::min(omega, rq.kmax) : omega;
    const pv_status st = (cap <= top) ? PV_EBUFSIZE : (any_ovf ? PV_EOVERFLOW : PV_OK);
    record_run(g, rq, st);
    return st;
}

extern "C" pv_status pv_local_frequency(pv_ctx *c, const pv_u128 *local, int64_t rows, int32_t K, int32_t col,
                                        pv_u128 *values, uint64_t *freq, int64_t cap, int64_t *ndistinct) {
    if (!c || rows < 0 || rows > INT32_MAX - 1 || K < 1 || col < 0 || col >= K || cap < 0 || !ndistinct ||
        (rows > 0 && !local) || (cap > 0 && (!values || !freq)))
        return PV_EINVAL;
    if (rows > 0) PVCHK(require_device(c->device, local, "local"));
    HIPCHK(hipSetDevice(c->device));
    BudgetScope scope(c);
    hipStream_t s = c->stream;
    const int n = (int)rows;
    long long npad = 1;
    while (npad < rows) npad <<= 1;
    PVCHK(c->ws.fq_keys.ensure((size_t)npad * 2));
    PVCHK(c->ws.fq_vals.ensure((size_t)std::max(n, 1) * 2));
    PVCHK(c->ws.fq_flags.ensure((size_t)n + 1));
    PVCHK(c->ws.fq_idx.ensure((size_t)n + 1));
    PVCHK(c->ws.fq_pos.ensure((size_t)n + 1));
    PVCHK(c->ws.scan.ensure((size_t)n / 1024 + 2));
    const FreqWork w{c->ws.fq_keys.p, c->ws.fq_vals.p, c->ws.fq_flags.p, c->ws.fq_idx.p, c->ws.fq_pos.p,
                     c->ws.scan.p};
    HIPCHK(pv_launch_frequency((const uint64_t *)local, n, K, col, npad, w, s));
    int D = 0;
    if (n > 0) HIPCHK(hipMemcpyAsync(&D, c->ws.fq_idx.p + n, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *ndistinct = D;
    if (cap < D) return PV_EBUFSIZE;
    if (D > 0) {
        std::vector<int> pos((size_t)D);
        HIPCHK(hipMemcpyAsync(values, c->ws.fq_vals.p, (size_t)D * 16, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(pos.data(), c->ws.fq_pos.p, (size_t)D * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int d = 0; d < D; d++) freq[d] = (uint64_t)((d + 1 < D ? pos[d + 1] : n) - pos[d]);
    }
    return PV_OK;
}

// The same without allocating: every intermediate lives in the device's
// static scratch array (its address resolved at pv_init), the
// multiplicities are formed on the device, and the results are copied
// straight into the caller's arrays.
extern "C" pv_status pv_local_frequency_static(pv_ctx *c, const pv_u128 *local, int64_t rows, int32_t K,
                                               int32_t col, pv_u128 *values, uint64_t *freq, int64_t cap,
                                               int64_t *ndistinct) {
    if (!c || rows < 0 || K < 1 || col < 0 || col >= K || cap < 0 || !ndistinct || (rows > 0 && !local) ||
        (cap > 0 && (!values || !freq)))
        return PV_EINVAL;
    if (rows > 0) PVCHK(require_device(c->device, local, "local"));
    if (rows > PV_FREQ_STATIC_ROWS) {
        snprintf(g_last_error, sizeof g_last_error, "%lld rows exceed the static scratch of %d rows",
                 (long long)rows, PV_FREQ_STATIC_ROWS);
        return PV_ETOOBIG;
    }
    HIPCHK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const int n = (int)rows;
    long long npad = 1;
    while (npad < rows) npad <<= 1;
    uint64_t *dvals = nullptr, *dfreq = nullptr;
    int *didx = nullptr;
    HIPCHK(pv_launch_frequency_static(c->device, (const uint64_t *)local, n, K, col, npad, &dvals, &dfreq, &didx,
                                      s));
    int D = 0;
    if (n > 0) HIPCHK(hipMemcpyAsync(&D, didx + n, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *ndistinct = D;
    if (cap < D) return PV_EBUFSIZE;
    if (D > 0) {
        HIPCHK(hipMemcpyAsync(values, dvals, (size_t)D * 16, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(freq, dfreq, (size_t)D * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    return PV_OK;
}

extern "C" pv_status pv_count_local(pv_graph *g, int32_t kind, int32_t k_lo, int32_t k_hi,
                                    pv_u128 *out, int64_t out_len, uint64_t *overflow_bits,
                                    pv_stats *stats) {
    if (!g || !out) return PV_EINVAL;
    if (kind != PV_VERTEX && kind != PV_EDGE) return PV_EINVAL;
    if (k_lo < 1 || k_hi < k_lo || k_hi > PV_MAX_ALPHA + 1) return PV_EINVAL;
    const int K = k_hi - k_lo + 1;
    const long long rows = (kind == PV_EDGE) ? g->nnz / 2 : (long long)g->n;
    const long long need = rows * K;
    if (out_len < need) return PV_EBUFSIZE;
    pv_ctx *c = g->ctx;
    GraphUse use(g);
    BudgetScope scope(c);
    PVCHK(prepare(g, false));
    PVCHK(c->ws.vout_own.ensure((size_t)std::max<long long>(need, 1) * 2));
    // k ranges wider than one pass's slots (16 per vertex, 8 per edge) are
    // counted window by window, each pass walking the tree truncated at its
    // own k_hi and writing its columns of the [rows][K] output
    const int win = (kind == PV_EDGE) ? 8 : PV_MAX_LOCAL_K;
    uint64_t lovf = 0;
    for (int w0 = k_lo; w0 <= k_hi; w0 += win) {
        const int w1 = std::min(k_hi, w0 + win - 1);
        CountReq rq;
        rq.kmax = w1;
        rq.what = "local";
        PVCHK(setup_local(g, kind, w0, w1, rq));
        rq.vout = c->ws.vout_own.p + 2 * (w0 - k_lo);
        rq.kstride = K;
        rq.order = g->order.p;
        rq.nheavy = g->nheavy;
        rq.nlight = g->nnonzero - g->nheavy;
        PVCHK(run_sct(g, rq));
        uint64_t wovf = 0;
        pv_status st = finish_counts(g, rq, nullptr, 0, nullptr, nullptr, stats, &wovf);
        if (st != PV_OK && st != PV_EOVERFLOW) return st;
        lovf |= wovf;
    }
    if (need)
        HIPCHK(hipMemcpyAsync(out, c->ws.vout_own.p, (size_t)need * 16, hipMemcpyDeviceToHost,
                              g->ctx->stream));
    HIPCHK(hipStreamSynchronize(g->ctx->stream));
    if (overflow_bits) overflow_bits[0] = lovf;
    return lovf ? PV_EOVERFLOW : PV_OK;
}

extern "C" pv_status pv_count_roots(pv_graph *g, const int32_t *roots, int32_t nroots, int32_t k_max,
                                    pv_u128 *counts, int32_t cap, int32_t *omega_out,
                                    uint64_t *overflow_bits, int32_t local_kind, int32_t k_lo, int32_t k_hi,
                                    pv_u128 *local_out, uint64_t *local_ovf, pv_stats *stats) {
    if (!g || nroots < 0 || (nroots > 0 && !roots) || cap < 0 || (cap > 0 && !counts))
        return PV_EINVAL;
    if (local_kind != PV_NONE && !local_out) return PV_EINVAL;
    if (local_kind != PV_NONE) PVCHK(require_device(g->ctx->device, local_out, "local_out"));
    if (local_ovf) *local_ovf = 0;
    GraphUse use(g);
    BudgetScope scope(g->ctx);
    PVCHK(prepare(g, false));
    // out-degrees of the chosen roots, heavy first (host-side scheduling only)
    std::vector<int> od(g->n);
    if (g->n) {
        HIPCHK(hipMemcpyAsync(od.data(), g->odeg.p, sizeof(int) * (size_t)g->n, hipMemcpyDeviceToHost,
                              g->ctx->stream));
        HIPCHK(hipStreamSynchronize(g->ctx->stream));
    }
    std::vector<int> rs;
    rs.reserve(nroots);
    std::vector<uint8_t> seen(g->n, 0);
    for (int i = 0; i < nroots; i++) {
        if (roots[i] < 0 || roots[i] >= g->n || seen[roots[i]]) return PV_EINVAL;
        seen[roots[i]] = 1;
        rs.push_back(roots[i]);
    }
    std::stable_sort(rs.begin(), rs.end(), [&](int a, int b) { return od[a] > od[b]; });
    int nheavy = 0;
    for (int v : rs) nheavy += (od[v] > PV_LIGHT_MAX) ? 1 : 0;
    DBuf<int> dorder;
    PVCHK(dorder.ensure(std::max<size_t>(rs.size(), 1)));
    if (!rs.empty()) {
        HIPCHK(hipMemcpyAsync(dorder.p, rs.data(), sizeof(int) * rs.size(), hipMemcpyHostToDevice,
                              g->ctx->stream));
    }
    CountReq rq;
    rq.kmax = k_max > 0 ? k_max : 0;
    rq.c0 = 0;
    rq.whole = false;
    rq.what = "roots";
    PVCHK(setup_local(g, local_kind, k_lo, k_hi, rq));
    rq.vout = (uint64_t *)local_out;
    rq.order = dorder.p;
    rq.nheavy = nheavy;
    rq.nlight = (int)rs.size() - nheavy;  // roots with an empty N+(v) are single leaves
    rq.size_n = (long long)rs.size();
    rq.size_m = 0;
    for (int v : rs) rq.size_m += od[v];
    pv_status st = run_sct(g, rq);
    if (st == PV_OK) st = finish_counts(g, rq, counts, cap, omega_out, overflow_bits, stats, local_ovf);
    dorder.release();
    return st;
}

extern "C" pv_status pv_graph_edge_list(pv_graph *g, int32_t *u, int32_t *v) {
    if (!g || ((!u || !v) && g->nnz > 0)) return PV_EINVAL;
    GraphUse use(g);
    HIPCHK(hipSetDevice(g->ctx->device));
    std::vector<int> rp((size_t)g->n + 1), col((size_t)std::max<long long>(g->nnz, 1));
    HIPCHK(hipMemcpyAsync(rp.data(), g->rp.p, sizeof(int) * rp.size(), hipMemcpyDeviceToHost,
                          g->ctx->stream));
    if (g->nnz)
        HIPCHK(hipMemcpyAsync(col.data(), g->col.p, sizeof(int) * (size_t)g->nnz,
                              hipMemcpyDeviceToHost, g->ctx->stream));
    HIPCHK(hipStreamSynchronize(g->ctx->stream));
    long long e = 0;
    for (int a = 0; a < g->n; a++)
        for (int i = rp[a]; i < rp[a + 1]; i++)
            if (col[i] > a) {
                u[e] = a;
                v[e] = col[i];
                e++;
            }
    return PV_OK;
}

extern "C" pv_status pv_count_batch(pv_ctx *c, int32_t G, pv_graph *const *gs, int32_t k_max,
                                    pv_u128 *counts, int32_t cap, int32_t *omega,
                                    uint64_t *overflow_bits, int32_t local_kind, int32_t k_lo,
                                    int32_t k_hi, pv_u128 *local_out, uint64_t *local_ovf,
                                    pv_status *status, pv_stats *stats) {
    if (!c || G < 0 || (G > 0 && (!gs || !counts)) || cap < 1) return PV_EINVAL;
    if (local_kind != PV_NONE && local_kind != PV_VERTEX) return PV_EINVAL;
    if (local_kind != PV_NONE && !local_out) return PV_EINVAL;
    if (local_kind != PV_NONE) PVCHK(require_device(c->device, local_out, "local_out"));
    if (local_ovf) *local_ovf = 0;
    if (G == 0) {
        if (stats) *stats = pv_stats{};
        return PV_OK;
    }
    HIPCHK(hipSetDevice(c->device));
    BudgetScope scope(c);
    // the member graphs are in use until the pass ends
    GraphUse use(gs, G);
    // the batch is counted as the disjoint union of its graphs
    std::vector<BatchPart> parts(G);
    long long N = 0, NNZ = 0;
    int maxdeg = 0;  // the union's largest degree (-1: some member's is not known)
    for (int b = 0; b < G; b++) {
        const pv_graph *g = gs[b];
        if (!g || g->ctx->device != c->device) return PV_EINVAL;
        maxdeg = (maxdeg < 0 || g->maxdeg < 0) ? -1 : std::max(maxdeg, g->maxdeg);
        parts[b].rp = g->rp.p;
        parts[b].col = g->col.p;
        parts[b].n = g->n;
        parts[b].voff = (int)N;
        parts[b].eoff = NNZ;
        parts[b].nnz = g->nnz;
        N += g->n;
        NNZ += g->nnz;
    }
    if (N >= (1ll << 30) || NNZ >= (1ll << 31)) return PV_ETOOBIG;
    if (!c->batch) PVCHK(graph_new(c, 0, 0, &c->batch));
    pv_graph *u = c->batch;
    u->n = (int)N;
    u->nnz = NNZ;
    u->maxdeg = maxdeg;
    u->oriented = false;
    u->eids = false;
    PVCHK(u->rp.ensure((size_t)N + 1));
    PVCHK(u->col.ensure((size_t)std::max<long long>(NNZ, 1)));
    PVCHK(u->vgraph.ensure((size_t)std::max<long long>(N, 1)));
    PVCHK(c->parts.ensure(G));
    hipStream_t s = c->stream;
    HIPCHK(hipMemcpyAsync(c->parts.p, parts.data(), sizeof(BatchPart) * G, hipMemcpyHostToDevice, s));
    HIPCHK(pv_launch_concat(c->parts.p, G, 0, u->rp.p, u->col.p, u->vgraph.p, s));
    const int nnz32 = (int)NNZ;  // the union's row_ptr[N] (a blocking copy: the source is on the stack)
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(u->rp.p + N, &nnz32, sizeof(int), hipMemcpyHostToDevice));
    PVCHK(prepare(u, true));
    u->deg_key.clear();  // a new union
    std::unique_ptr<TuneScope> tuned;
    PVCHK(tune_scope_for(u, local_kind, k_lo, k_hi, k_max, tuned));
    CountReq rq;
    rq.kmax = k_max > 0 ? k_max : 0;
    PVCHK(setup_local(u, local_kind, k_lo, k_hi, rq));
    rq.vout = (uint64_t *)local_out;
    rq.graphs = G;
    rq.what = "batch";
    rq.vgraph = u->vgraph.p;
    rq.order = u->order.p;
    rq.nheavy = u->nheavy;
    rq.nlight = u->nnonzero - u->nheavy;
    PVCHK(run_sct(u, rq));
    return finish_counts(u, rq, counts, cap, omega, overflow_bits, stats, local_ovf, status);
}

extern "C" pv_status pv_count_global_batch(pv_ctx *c, int32_t G, pv_graph *const *gs, int32_t k_max,
                                           pv_u128 *counts, int32_t cap, int32_t *omega,
                                           uint64_t *overflow_bits, pv_status *status, pv_stats *stats) {
    return pv_count_batch(c, G, gs, k_max, counts, cap, omega, overflow_bits, PV_NONE, 0, 0, nullptr,
                          nullptr, status, stats);
}

// ------------------------------------------------------------- tuning
// The settings that split the walk (dfs_max, dfs_budget, lane_max) change
// neither the tree nor the counts, only how the work lands on the device.
// pv_autotune times candidates on a graph and keeps the fastest under a key
// made of the device, the kind of count and the graph's out-degree
// histogram (powers of two, each count rounded to its power of two), so
// graphs of the same shape share an entry.

static std::string mode_key(int kind, int klo, int khi, int kmax) {
    std::string m = kind == PV_VERTEX ? "v" : (kind == PV_EDGE ? "e" : "g");
    if (kind != PV_NONE) m += std::to_string(khi - klo + 1);
    if (kmax > 0) m += "t" + std::to_string(kmax);
    return m;
}

// the out-degree histogram part of g's key (g oriented)
static pv_status deg_key_of(pv_graph *g) {
    if (!g->deg_key.empty()) return PV_OK;
    pv_ctx *c = g->ctx;
    DBuf<int> dh;
    PVCHK(dh.ensure(PV_DEG_BUCKETS));
    HIPCHK(hipMemsetAsync(dh.p, 0, PV_DEG_BUCKETS * sizeof(int), c->stream));
    HIPCHK(pv_launch_deg_hist(g->n, g->odeg.p, dh.p, c->stream));
    int h[PV_DEG_BUCKETS];
    hipError_t e = hipMemcpyAsync(h, dh.p, sizeof h, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dh.release();
    if (e != hipSuccess) {
        set_err("deg_key_of", e);
        return PV_EDEVICE;
    }
    std::string k = "h";
    for (int b = 0; b < PV_DEG_BUCKETS; b++) {
        const unsigned x = (unsigned)h[b];
        k += std::to_string(x ? 32 - __builtin_clz(x) : 0);
        if (b + 1 < PV_DEG_BUCKETS) k += ".";
    }
    g->deg_key = k;
    return PV_OK;
}

static std::string full_key(const pv_graph *g, const std::string &mode) {
    return g->ctx->arch + "|" + mode + "|" + g->deg_key;
}

// the tuned settings of a key for the duration of one call
TuneScope::TuneScope(pv_ctx *c_, const std::string &key) : c(c_) {
    auto it = c->tune.find(key);
    if (it == c->tune.end()) return;
    on = true;
    dm = c->dfs_max;
    db = c->dfs_budget;
    lm = c->lane_max;
    c->dfs_max = it->second.dfs_max;
    c->dfs_budget = it->second.dfs_budget;
    c->lane_max = it->second.lane_max;
}

TuneScope::~TuneScope() {
    if (!on) return;
    c->dfs_max = dm;
    c->dfs_budget = db;
    c->lane_max = lm;
}

static pv_status tune_scope_for(pv_graph *g, int kind, int klo, int khi, int kmax,
                                std::unique_ptr<TuneScope> &scope) {
    if (g->ctx->tune.empty()) return PV_OK;
    PVCHK(deg_key_of(g));
    scope.reset(new (std::nothrow) TuneScope(g->ctx, full_key(g, mode_key(kind, klo, khi, kmax))));
    return PV_OK;
}

// numbers and strings after `"name":` inside one JSON object of the cache
static bool json_num(const std::string &obj, const char *name, double &v) {
    const std::string pat = std::string("\"") + name + "\"";
    size_t i = obj.find(pat);
    if (i == std::string::npos) return false;
    i = obj.find(':', i + pat.size());
    if (i == std::string::npos) return false;
    char *end = nullptr;
    v = strtod(obj.c_str() + i + 1, &end);
    return end != obj.c_str() + i + 1;
}

static bool json_str(const std::string &obj, const char *name, std::string &v) {
    const std::string pat = std::string("\"") + name + "\"";
    size_t i = obj.find(pat);
    if (i == std::string::npos) return false;
    i = obj.find('"', obj.find(':', i + pat.size()));
    if (i == std::string::npos) return false;
    const size_t j = obj.find('"', i + 1);
    if (j == std::string::npos) return false;
    v = obj.substr(i + 1, j - i - 1);
    return true;
}

static void tune_load(pv_ctx *c) {
    std::ifstream f(c->tune_path);
    if (!f) return;  // no cache yet: pv_autotune creates it
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string txt = ss.str();
    size_t pos = txt.find("\"entries\"");
    while (pos != std::string::npos) {
        const size_t a = txt.find('{', pos + 1);
        if (a == std::string::npos) break;
        const size_t b = txt.find('}', a);
        if (b == std::string::npos) break;
        const std::string obj = txt.substr(a, b - a + 1);
        std::string key;
        double dm, db, lm, mb = 0, md = 0;
        if (json_str(obj, "key", key) && json_num(obj, "dfs_max", dm) && json_num(obj, "dfs_budget", db) &&
            json_num(obj, "lane_max", lm) && dm >= 1 && dm <= 64 && (db == 0 || (db >= 16 && db <= (1 << 20))) &&
            lm >= 0 && lm <= PV_LANE_MAX) {
            json_num(obj, "ms_best", mb);
            json_num(obj, "ms_default", md);
            TuneEntry e;
            e.dfs_max = (int)dm;
            e.dfs_budget = (int)db;
            e.lane_max = (int)lm;
            e.ms_best = (float)mb;
            e.ms_default = (float)md;
            c->tune[key] = e;
        }
        pos = b;
    }
}

static pv_status tune_save(pv_ctx *c) {
    if (c->tune_path.empty()) return PV_OK;
    const std::string tmp = c->tune_path + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) {
            snprintf(g_last_error, sizeof g_last_error, "cannot write %s", tmp.c_str());
            return PV_EINVAL;
        }
        f << "{\n  \"entries\": [\n";
        size_t i = 0;
        for (const auto &kv : c->tune) {
            char line[256];
            snprintf(line, sizeof line,
                     "\"dfs_max\": %d, \"dfs_budget\": %d, \"lane_max\": %d, \"ms_best\": %.4f, \"ms_default\": %.4f",
                     kv.second.dfs_max, kv.second.dfs_budget, kv.second.lane_max, kv.second.ms_best,
                     kv.second.ms_default);
            f << "    {\"key\": \"" << kv.first << "\", " << line << "}" << (++i < c->tune.size() ? "," : "")
              << "\n";
        }
        f << "  ]\n}\n";
    }
    if (rename(tmp.c_str(), c->tune_path.c_str()) != 0) {
        snprintf(g_last_error, sizeof g_last_error, "cannot replace %s", c->tune_path.c_str());
        return PV_EINVAL;
    }
    return PV_OK;
}

extern "C" const char *pv_tune_key(pv_graph *g, int32_t local_kind, int32_t k_lo, int32_t k_hi) {
    static thread_local std::string key;
    key.clear();
    if (!g) return "";
    BudgetScope scope(g->ctx);
    if (prepare(g, false) != PV_OK || deg_key_of(g) != PV_OK) return "";
    key = full_key(g, mode_key(local_kind, k_lo, k_hi, 0));
    return key.c_str();
}

extern "C" pv_status pv_autotune(pv_graph *g, int32_t local_kind, int32_t k_lo, int32_t k_hi,
                                 pv_u128 *local_out, int32_t reps, pv_tune *out) {
    if (!g || reps < 1 || (local_kind != PV_NONE && !local_out)) return PV_EINVAL;
    pv_ctx *c = g->ctx;
    {
        GraphUse use(g);
        BudgetScope scope(c);
        PVCHK(prepare(g, false));
        PVCHK(deg_key_of(g));
    }
    const std::string key = full_key(g, mode_key(local_kind, k_lo, k_hi, 0));
    const int dm0 = c->dfs_max, db0 = c->dfs_budget, lm0 = c->lane_max;
    std::vector<pv_u128> counts(PV_MAX_ALPHA + 2);
    int trials = 0;
    auto time_of = [&](int dm, int db, int lm, float &ms) -> pv_status {
        c->dfs_max = dm;
        c->dfs_budget = db;
        c->lane_max = lm;
        ms = 1e30f;
        for (int r = 0; r < reps; r++) {
            const auto t0 = std::chrono::steady_clock::now();
            pv_status st = count_untuned(g, 0, 0, counts.data(), (int)counts.size(), nullptr, nullptr, local_kind,
                                         k_lo, k_hi, local_out, nullptr, nullptr);
            if (st != PV_OK && st != PV_EOVERFLOW) return st;
            const float t = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
            ms = std::min(ms, t);
        }
        trials++;
        return PV_OK;
    };
    TuneEntry best;
    best.dfs_max = dm0;
    best.dfs_budget = db0;
    best.lane_max = lm0;
    pv_status st = time_of(dm0, db0, lm0, best.ms_default);
    best.ms_best = best.ms_default;
    // one setting at a time from the current best
    static const int LANES[] = {0, 4, 6, 8};
    static const int BUDGETS[] = {0, 1024, 2048, 4096, 8192, 16384};
    static const int DMAX[] = {32, 48, 64};
    for (int pass = 0; pass < 3 && st == PV_OK; pass++) {
        const int *vals = pass == 0 ? LANES : (pass == 1 ? BUDGETS : DMAX);
        const int nv = pass == 0 ? 4 : (pass == 1 ? 6 : 3);
        for (int i = 0; i < nv && st == PV_OK; i++) {
            TuneEntry e = best;
            int &slot = pass == 0 ? e.lane_max : (pass == 1 ? e.dfs_budget : e.dfs_max);
            if (slot == vals[i]) continue;
            slot = vals[i];
            float ms = 0.f;
            st = time_of(e.dfs_max, e.dfs_budget, e.lane_max, ms);
            if (st == PV_OK && ms < best.ms_best) {
                best.dfs_max = e.dfs_max;
                best.dfs_budget = e.dfs_budget;
                best.lane_max = e.lane_max;
                best.ms_best = ms;
            }
        }
    }
    c->dfs_max = dm0;
    c->dfs_budget = db0;
    c->lane_max = lm0;
    if (st != PV_OK) return st;
    c->tune[key] = best;
    PVCHK(tune_save(c));
    if (out) {
        out->dfs_max = best.dfs_max;
        out->dfs_budget = best.dfs_budget;
        out->lane_max = best.lane_max;
        out->ms_best = best.ms_best;
        out->ms_default = best.ms_default;
        out->trials = trials;
    }
    return PV_OK;
}
