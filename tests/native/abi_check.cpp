// A native check of the C ABI, built with the host sanitizers (AddressSanitizer
// and UndefinedBehaviorSanitizer on the library's host code and on this file)
// and with the library's device-side invariant checks on (PV_CHECKED).  It
// drives every entry point family on small graphs whose counts are known:
// complete graphs (C_k = C(n, k), c_k(v) = C(n-1, k-1), c_k(e) = C(n-2, k-2)),
// paths, complete multipartite graphs (C_k = e_k of the part sizes), and
// random graphs of at most 64 vertices against a brute-force enumeration of
// their cliques.  Error paths: malformed input, null pointers, small buffers.
//
// Exit status: 0 all checks passed, 1 a check failed, 77 no HIP device.
#include <hip/hip_runtime_api.h>
#include <pivoter.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace {

int g_checks = 0, g_failed = 0;

#define CHECK(cond, ...)                                          \
    do {                                                          \
        g_checks++;                                               \
        if (!(cond)) {                                            \
            g_failed++;                                           \
            fprintf(stderr, "FAILED %s:%d: ", __FILE__, __LINE__); \
            fprintf(stderr, __VA_ARGS__);                         \
            fprintf(stderr, " [%s]\n", pv_last_error());          \
        }                                                         \
    } while (0)

#define OK(call) CHECK((call) == PV_OK, "%s", #call)

using u128 = unsigned __int128;

u128 val(const pv_u128 &x) { return ((u128)x.hi << 64) | x.lo; }

// binomials by Pascal's rule (every C(n, k) with n <= 130 fits 128 bits)
u128 binom(int n, int k) {
    static std::vector<std::vector<u128>> t;
    if (t.empty()) {
        t.assign(131, std::vector<u128>(131, 0));
        for (int a = 0; a <= 130; a++) {
            t[a][0] = 1;
            for (int b = 1; b <= a; b++) t[a][b] = t[a - 1][b - 1] + (b < a ? t[a - 1][b] : 0);
        }
    }
    if (k < 0 || n < 0 || k > n || n > 130) return 0;
    return t[n][k];
}

struct Graph {
    int n = 0;
    std::vector<int32_t> rp{0}, col;
};

Graph from_adj(int n, const std::vector<uint64_t> &adj) {
    Graph g;
    g.n = n;
    g.rp.assign(1, 0);
    for (int v = 0; v < n; v++) {
        for (int u = 0; u < n; u++)
            if ((adj[v] >> u) & 1) g.col.push_back(u);
        g.rp.push_back((int32_t)g.col.size());
    }
    return g;
}

Graph complete(int n) {
    Graph g;
    g.n = n;
    for (int v = 0; v < n; v++) {
        for (int u = 0; u < n; u++)
            if (u != v) g.col.push_back(u);
        g.rp.push_back((int32_t)g.col.size());
    }
    return g;
}

Graph path(int n) {
    Graph g;
    g.n = n;
    for (int v = 0; v < n; v++) {
        if (v > 0) g.col.push_back(v - 1);
        if (v + 1 < n) g.col.push_back(v + 1);
        g.rp.push_back((int32_t)g.col.size());
    }
    return g;
}

// complete multipartite graph with parts of the given sizes
Graph multipartite(const std::vector<int> &parts) {
    std::vector<int> part;
    for (size_t i = 0; i < parts.size(); i++) part.insert(part.end(), parts[i], (int)i);
    Graph g;
    g.n = (int)part.size();
    for (int v = 0; v < g.n; v++) {
        for (int u = 0; u < g.n; u++)
            if (part[u] != part[v]) g.col.push_back(u);
        g.rp.push_back((int32_t)g.col.size());
    }
    return g;
}

// G(n, p) from a 64-bit linear congruential generator (Knuth's MMIX constants)
std::vector<uint64_t> random_adj(int n, double p, uint64_t seed) {
    std::vector<uint64_t> adj(n, 0);
    uint64_t x = seed * 2862933555777941757ull + 3037000493ull;
    for (int v = 0; v < n; v++)
        for (int u = v + 1; u < n; u++) {
            x = x * 6364136223846793005ull + 1442695040888963407ull;
            if ((double)(x >> 11) * (1.0 / 9007199254740992.0) < p) {
                adj[v] |= 1ull << u;
                adj[u] |= 1ull << v;
            }
        }
    return adj;
}

// every clique of a graph on at most 64 vertices, by extending with larger
// ids only: global counts, per-vertex counts and per-edge counts (edge id =
// rank of (u, v), u < v, in lexicographic order)
struct Brute {
    int n;
    const std::vector<uint64_t> &adj;
    std::vector<uint64_t> glob;
    std::vector<std::vector<uint64_t>> vert, edge;
    std::vector<int> eid;  // u * 64 + v -> edge id
    std::vector<int> members;
    Brute(int n_, const std::vector<uint64_t> &a) : n(n_), adj(a), glob(66, 0), vert(n_, std::vector<uint64_t>(66, 0)),
                                                  eid(64 * 64, -1) {
        int m = 0;
        for (int u = 0; u < n; u++)
            for (int v = u + 1; v < n; v++)
                if ((adj[u] >> v) & 1) eid[u * 64 + v] = m++;
        edge.assign(m, std::vector<uint64_t>(66, 0));
        glob[0] = 1;
        rec(n ? (~0ull >> (64 - n)) : 0ull);
    }
    void rec(uint64_t cand) {
        while (cand) {
            const int v = __builtin_ctzll(cand);
            cand &= cand - 1;
            members.push_back(v);
            const int k = (int)members.size();
            glob[k]++;
            for (int x : members) vert[x][k]++;
            for (int i = 0; i < k; i++)
                for (int j = i + 1; j < k; j++) {
                    const int a = std::min(members[i], members[j]), b = std::max(members[i], members[j]);
                    edge[eid[a * 64 + b]][k]++;
                }
            rec(cand & adj[v]);
            members.pop_back();
        }
    }
};

pv_graph *load(pv_ctx *c, const Graph &g, uint32_t flags = 0) {
    pv_graph *h = nullptr;
    const pv_status s = pv_graph_load_csr(c, g.n, g.rp.data(), g.col.data(), flags, &h);
    CHECK(s == PV_OK && h, "load n=%d", g.n);
    return s == PV_OK ? h : nullptr;
}

void check_global(pv_graph *h, const std::vector<u128> &want, const char *what) {
    std::vector<pv_u128> c(PV_MAX_ALPHA + 2);
    int32_t omega = -1;
    uint64_t ovf[(PV_MAX_ALPHA + 2 + 63) / 64] = {};
    pv_stats st;
    const pv_status s = pv_count_global(h, 0, c.data(), (int32_t)c.size(), &omega, ovf, &st);
    CHECK(s == PV_OK, "%s: pv_count_global status %d", what, s);
    if (s != PV_OK) return;
    int top = 0;
    for (size_t k = 0; k < want.size(); k++)
        if (want[k]) top = (int)k;
    CHECK(omega == top, "%s: omega %d, want %d", what, omega, top);
    for (size_t k = 0; k < c.size(); k++) {
        const u128 w = k < want.size() ? want[k] : 0;
        if (val(c[k]) != w) {
            CHECK(false, "%s: C_%zu differs", what, k);
            return;
        }
    }
}

void check_complete(pv_ctx *c, int n) {
    char what[64];
    snprintf(what, sizeof what, "K_%d", n);
    pv_graph *h = load(c, complete(n));
    if (!h) return;
    std::vector<u128> want(n + 1);
    for (int k = 0; k <= n; k++) want[k] = binom(n, k);
    check_global(h, want, what);
    pv_stats st;
    std::vector<pv_u128> cc(n + 2);
    int32_t om;
    uint64_t ovf[4] = {};
    OK(pv_count_global(h, 0, cc.data(), n + 2, &om, ovf, &st));
    // one pivot chain per root: a leaf per vertex, n(n+1)/2 nodes
    CHECK(st.leaves == (uint64_t)n && st.nodes == (uint64_t)n * (n + 1) / 2, "%s: tree %llu nodes %llu leaves", what,
          (unsigned long long)st.nodes, (unsigned long long)st.leaves);
    if (n >= 3 && n <= 40) {
        const int klo = 1, khi = std::min(n, 8), K = khi - klo + 1;
        std::vector<pv_u128> vo((size_t)n * K), eo((size_t)n * (n - 1) / 2 * K);
        uint64_t lov = 0;
        OK(pv_count_local(h, PV_VERTEX, klo, khi, vo.data(), (int64_t)vo.size(), &lov, &st));
        bool good = lov == 0;
        for (int v = 0; v < n; v++)
            for (int k = klo; k <= khi; k++) good = good && val(vo[(size_t)v * K + (k - klo)]) == binom(n - 1, k - 1);
        CHECK(good, "%s: per-vertex counts", what);
        const int ehi = std::min(n, 8), EK = ehi - 2 + 1;
        std::vector<pv_u128> e2((size_t)n * (n - 1) / 2 * EK);
        OK(pv_count_local(h, PV_EDGE, 2, ehi, e2.data(), (int64_t)e2.size(), &lov, &st));
        good = lov == 0;
        for (size_t e = 0; e < (size_t)n * (n - 1) / 2; e++)
            for (int k = 2; k <= ehi; k++) good = good && val(e2[e * EK + (k - 2)]) == binom(n - 2, k - 2);
        CHECK(good, "%s: per-edge counts", what);
        // frequency distributions of a device table of local counts: every
        // vertex of K_n has the same count, so each column has one value
        pv_u128 *d = nullptr;
        CHECK(hipMalloc((void **)&d, vo.size() * sizeof(pv_u128)) == hipSuccess, "hipMalloc");
        if (d) {
            CHECK(hipMemcpy(d, vo.data(), vo.size() * sizeof(pv_u128), hipMemcpyHostToDevice) == hipSuccess, "copy");
            for (int col = 0; col < K; col++) {
                pv_u128 values[2];
                uint64_t freq[2];
                int64_t nd = -1;
                OK(pv_local_frequency(c, d, n, K, col, values, freq, 2, &nd));
                CHECK(nd == 1 && freq[0] == (uint64_t)n && val(values[0]) == binom(n - 1, col + klo - 1),
                      "%s: frequencies of column %d", what, col);
                nd = -1;
                OK(pv_local_frequency_static(c, d, n, K, col, values, freq, 2, &nd));
                CHECK(nd == 1 && freq[0] == (uint64_t)n && val(values[0]) == binom(n - 1, col + klo - 1),
                      "%s: frequencies of column %d (no allocation)", what, col);
            }
            int64_t nd = -1;
            OK(pv_local_frequency(c, nullptr, 0, K, 0, nullptr, nullptr, 0, &nd));
            CHECK(nd == 0, "%s: frequency of no rows", what);
            CHECK(hipFree(d) == hipSuccess, "hipFree");
        }
    }
    OK(pv_graph_free(h));
}

void check_random(pv_ctx *c, int n, double p, uint64_t seed) {
    char what[64];
    snprintf(what, sizeof what, "G(%d, %.2f) seed %llu", n, p, (unsigned long long)seed);
    const std::vector<uint64_t> adj = random_adj(n, p, seed);
    const Graph g = from_adj(n, adj);
    const Brute b(n, adj);
    pv_graph *h = load(c, g);
    if (!h) return;
    std::vector<u128> want(b.glob.begin(), b.glob.end());
    check_global(h, want, what);
    int omega = 0;
    for (int k = 0; k < 66; k++)
        if (b.glob[k]) omega = k;
    const int klo = 1, khi = std::max(1, std::min(omega, 16)), K = khi - klo + 1;
    std::vector<pv_u128> vo((size_t)n * K);
    uint64_t lov = 0;
    pv_stats st;
    OK(pv_count_local(h, PV_VERTEX, klo, khi, vo.data(), (int64_t)vo.size(), &lov, &st));
    bool good = lov == 0;
    for (int v = 0; v < n; v++)
        for (int k = klo; k <= khi; k++) good = good && val(vo[(size_t)v * K + (k - klo)]) == b.vert[v][k];
    CHECK(good, "%s: per-vertex counts", what);
    const size_t m = b.edge.size();
    if (m > 0 && omega >= 2) {
        const int ehi = std::min(omega, 9), EK = ehi - 2 + 1;
        std::vector<pv_u128> eo(m * EK);
        OK(pv_count_local(h, PV_EDGE, 2, ehi, eo.data(), (int64_t)eo.size(), &lov, &st));
        good = lov == 0;
        for (size_t e = 0; e < m; e++)
            for (int k = 2; k <= ehi; k++) good = good && val(eo[e * EK + (k - 2)]) == b.edge[e][k];
        CHECK(good, "%s: per-edge counts", what);
        std::vector<int32_t> eu(m), ev(m);
        OK(pv_graph_edge_list(h, eu.data(), ev.data()));
        good = true;
        for (size_t e = 0; e < m; e++) good = good && eu[e] < ev[e] && b.eid[eu[e] * 64 + ev[e]] == (int)e;
        CHECK(good, "%s: edge list order", what);
    }
    // a root subset and its complement add up to the whole
    std::vector<int32_t> r1, r2;
    for (int v = 0; v < n; v++) (v % 3 ? r1 : r2).push_back(v);
    std::vector<pv_u128> c1(70), c2(70), v1((size_t)n * K), v2((size_t)n * K);
    int32_t o1, o2;
    uint64_t ov1[2] = {}, ov2[2] = {}, l1 = 0, l2 = 0;
    // local output of a root subset goes to device memory; a host buffer is refused
    CHECK(pv_count_roots(h, r1.data(), (int32_t)r1.size(), 0, c1.data(), 70, &o1, ov1, PV_VERTEX, klo, khi, v1.data(),
                         &l1, &st) == PV_EINVAL,
          "%s: host local_out refused", what);
    pv_u128 *d1 = nullptr, *d2 = nullptr;
    const size_t bytes = v1.size() * sizeof(pv_u128);
    CHECK(hipMalloc((void **)&d1, bytes) == hipSuccess && hipMalloc((void **)&d2, bytes) == hipSuccess, "hipMalloc");
    OK(pv_count_roots(h, r1.data(), (int32_t)r1.size(), 0, c1.data(), 70, &o1, ov1, PV_VERTEX, klo, khi, d1, &l1, &st));
    OK(pv_count_roots(h, r2.data(), (int32_t)r2.size(), 0, c2.data(), 70, &o2, ov2, PV_VERTEX, klo, khi, d2, &l2, &st));
    CHECK(hipMemcpy(v1.data(), d1, bytes, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(v2.data(), d2, bytes, hipMemcpyDeviceToHost) == hipSuccess,
          "copy back");
    (void)hipFree(d1);
    (void)hipFree(d2);
    good = true;
    for (int k = 1; k < 66; k++) good = good && val(c1[k]) + val(c2[k]) == (u128)b.glob[k];
    for (size_t i = 0; i < vo.size(); i++) good = good && val(v1[i]) + val(v2[i]) == val(vo[i]);
    CHECK(good, "%s: root subsets add up", what);
    // truncated counts: C_k for k <= k_max
    std::vector<pv_u128> ct(70);
    int32_t ot;
    uint64_t ovt[2] = {};
    const int kt = std::max(1, omega - 1);
    OK(pv_count_global(h, kt, ct.data(), 70, &ot, ovt, &st));
    good = true;
    for (int k = 1; k <= kt; k++) good = good && val(ct[k]) == (u128)b.glob[k];
    CHECK(good, "%s: counts truncated at k_max = %d", what, kt);
    OK(pv_graph_free(h));
}

void check_errors(pv_ctx *c) {
    pv_graph *h = nullptr;
    const int32_t rp_loop[3] = {0, 2, 3}, col_loop[3] = {0, 1, 0};  // self loop at 0
    CHECK(pv_graph_load_csr(c, 2, rp_loop, col_loop, 0, &h) == PV_ENOTSIMPLE, "self loop refused");
    const int32_t rp_asym[3] = {0, 1, 1}, col_asym[1] = {1};  // missing reverse edge
    CHECK(pv_graph_load_csr(c, 2, rp_asym, col_asym, 0, &h) == PV_ENOTSIMPLE, "asymmetric CSR refused");
    CHECK(pv_graph_load_csr(c, 2, rp_asym, col_asym, PV_SYMMETRIZE, &h) == PV_OK, "asymmetric CSR repaired");
    if (h) {
        std::vector<u128> want = {1, 2, 1};
        check_global(h, want, "repaired K_2");
        OK(pv_graph_free(h));
    }
    CHECK(pv_graph_load_csr(c, -1, rp_asym, col_asym, 0, &h) == PV_EINVAL, "negative n");
    CHECK(pv_graph_load_csr(nullptr, 2, rp_asym, col_asym, 0, &h) == PV_EINVAL, "null context");
    CHECK(pv_cancel(nullptr) == PV_EINVAL, "cancel without a context");
    h = load(c, complete(12));
    if (h) {
        pv_u128 small[4];
        int32_t om;
        uint64_t ov[1] = {};
        pv_stats st;
        CHECK(pv_count_global(h, 0, small, 4, &om, ov, &st) == PV_EBUFSIZE, "small count buffer");
        pv_u128 lo[4];
        uint64_t lov;
        CHECK(pv_count_local(h, PV_VERTEX, 1, 4, lo, 4, &lov, &st) == PV_EBUFSIZE, "small local buffer");
        CHECK(pv_count_local(h, PV_VERTEX, 5, 4, lo, 4, &lov, &st) == PV_EINVAL, "empty k range");
        CHECK(pv_count_local(h, 7, 1, 4, lo, 4, &lov, &st) == PV_EINVAL, "unknown local kind");
        OK(pv_graph_free(h));
    }
    for (pv_status s = 0; s >= -10; s--) CHECK(pv_strerror(s) && *pv_strerror(s), "strerror(%d)", s);
}

void check_batch(pv_ctx *c) {
    std::vector<Graph> gs = {complete(9), path(30), multipartite({3, 3, 3, 2}), Graph()};
    std::vector<pv_graph *> hs;
    for (const Graph &g : gs) hs.push_back(load(c, g));
    if (std::find(hs.begin(), hs.end(), nullptr) != hs.end()) return;
    const int G = (int)hs.size(), cap = 16;
    std::vector<pv_u128> counts((size_t)G * cap);
    std::vector<int32_t> omega(G);
    std::vector<uint64_t> ovf(G);
    std::vector<pv_status> st(G, -99);
    pv_stats stats;
    OK(pv_count_global_batch(c, G, hs.data(), 0, counts.data(), cap, omega.data(), ovf.data(), st.data(), &stats));
    std::vector<std::vector<u128>> want(G, std::vector<u128>(cap, 0));
    for (int k = 0; k <= 9; k++) want[0][k] = binom(9, k);
    want[1][0] = 1, want[1][1] = 30, want[1][2] = 29;
    // e_k(3, 3, 3, 2)
    const int parts[4] = {3, 3, 3, 2};
    std::vector<u128> e(5, 0);
    e[0] = 1;
    for (int x : parts)
        for (int k = 4; k >= 1; k--) e[k] += e[k - 1] * (u128)x;
    for (int k = 0; k <= 4; k++) want[2][k] = e[k];
    want[3][0] = 1;
    bool good = true;
    for (int b = 0; b < G; b++) {
        good = good && st[b] == PV_OK;
        for (int k = 0; k < cap; k++) good = good && val(counts[(size_t)b * cap + k]) == want[b][k];
    }
    CHECK(good, "batch of four graphs (one empty)");
    for (pv_graph *h : hs) OK(pv_graph_free(h));
}

void check_server() {
    pv_server_cfg cfg = {0, 2, 4, 64ll << 20, 256ll << 20};
    pv_server *srv = nullptr;
    OK(pv_server_start(&cfg, &srv));
    if (!srv) return;
    const Graph k10 = complete(10), p20 = path(20);
    std::vector<pv_u128> c1(16), c2(16), v2((size_t)20 * 2);
    pv_request r1 = {1, k10.n, k10.rp.data(), k10.col.data(), PV_REQ_GLOBAL, 0, 0, c1.data(), 16, nullptr};
    pv_request r2 = {2, p20.n, p20.rp.data(), p20.col.data(), PV_REQ_VERTEX, 1, 2, c2.data(), 16, v2.data()};
    uint64_t t1 = 0, t2 = 0;
    OK(pv_server_submit(srv, &r1, &t1));
    OK(pv_server_submit(srv, &r2, &t2));
    pv_result o1, o2;
    OK(pv_server_wait(srv, t1, -1, &o1));
    OK(pv_server_wait(srv, t2, -1, &o2));
    bool good = o1.status == PV_OK && o2.status == PV_OK;
    for (int k = 0; k <= 10; k++) good = good && val(c1[k]) == binom(10, k);
    good = good && val(c2[1]) == 20 && val(c2[2]) == 19 && val(c2[3]) == 0;
    for (int v = 0; v < 20; v++) good = good && val(v2[v * 2]) == 1 && val(v2[v * 2 + 1]) == (v == 0 || v == 19 ? 1u : 2u);
    CHECK(good, "served results");
    pv_server_stop(srv);
}

}  // namespace

int main() {
    pv_ctx *c = nullptr;
    pv_config cfg;
    memset(&cfg, 0, sizeof cfg);
    const pv_status s = pv_init(0, &cfg, &c);
    if (s != PV_OK) {
        printf("abi_check: no device (%s: %s)\n", pv_strerror(s), pv_last_error());
        return 77;
    }
    for (int n : {1, 2, 5, 20, 40, 64, 65, 130}) check_complete(c, n);
    check_random(c, 30, 0.3, 1);
    check_random(c, 48, 0.5, 2);
    check_random(c, 64, 0.7, 3);
    check_random(c, 64, 0.05, 4);
    // the same trees split into many units: level items, frame items and the
    // lane tier switched off, then on again
    OK(pv_set_dfs_max(c, 8));
    OK(pv_set_dfs_budget(c, 16));
    check_random(c, 64, 0.7, 5);
    OK(pv_set_lane_max(c, 0));
    check_random(c, 48, 0.5, 6);
    OK(pv_set_lane_max(c, 8));
    OK(pv_set_dfs_budget(c, 0));
    OK(pv_set_dfs_max(c, 64));
    check_errors(c);
    check_batch(c);
    {
        const std::vector<int> parts = {2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2};
        pv_graph *h = load(c, multipartite(parts));
        if (h) {
            std::vector<u128> want(13);
            for (int k = 0; k <= 12; k++) want[k] = binom(12, k) << k;
            check_global(h, want, "K_{2 x 12}");
            OK(pv_graph_free(h));
        }
    }
    int64_t held = -1;
    OK(pv_memory(c, &held));
    pv_fini(c);
    check_server();
    printf("abi_check: %d checks, %d failed\n", g_checks, g_failed);
    return g_failed ? 1 : 0;
}
