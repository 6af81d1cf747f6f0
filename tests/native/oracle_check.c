/*
 * The CPU oracle (oracle/oracle.c) run under AddressSanitizer and
 * UndefinedBehaviorSanitizer: every output of orc_count -- global, per-vertex
 * and per-edge counts, the leaf histogram, truncated counts and root
 * subsets -- on complete graphs (closed forms) and on random graphs of at
 * most 64 vertices against a brute-force enumeration of their cliques.
 * Exit status 0 when every check passes.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t orc_peel(int32_t n, const int32_t *rp, const int32_t *col, int32_t *sub, int32_t *alpha_out);
int32_t orc_count(int32_t n, const int32_t *rp, const int32_t *col, const int32_t *key_in, const int32_t *prio,
                  const int32_t *roots, int32_t nroots, int32_t kmax, int32_t kcap, uint64_t *glob, uint8_t *govf,
                  int32_t vlo, int32_t vhi, uint64_t *vc, uint8_t *vovf, int32_t elo, int32_t ehi, uint64_t *ec,
                  uint8_t *eovf, int32_t hd, uint64_t *hist, uint64_t *stats);

typedef unsigned __int128 u128;
static int checks, failed;

#define CHECK(cond, ...)                                                  \
    do {                                                                  \
        checks++;                                                         \
        if (!(cond)) {                                                    \
            failed++;                                                     \
            fprintf(stderr, "FAILED line %d: ", __LINE__);                \
            fprintf(stderr, __VA_ARGS__);                                 \
            fprintf(stderr, "\n");                                        \
        }                                                                 \
    } while (0)

static u128 pascal[131][131];

static u128 binom(int n, int k) { return (n < 0 || k < 0 || k > n || n > 130) ? 0 : pascal[n][k]; }

static u128 limbs(const uint64_t *x) { return ((u128)x[1] << 64) | x[0]; }

/* brute force over a graph of at most 64 vertices */
static int bn;
static const uint64_t *badj;
static uint64_t *bglob, *bvert, *bedge; /* [66], [n][66], [m][66] */
static int *beid;                        /* [64 * 64] */
static int memb[64], depth;

static void rec(uint64_t cand) {
    while (cand) {
        const int v = __builtin_ctzll(cand);
        cand &= cand - 1;
        memb[depth++] = v;
        const int k = depth;
        bglob[k]++;
        for (int i = 0; i < k; i++) bvert[memb[i] * 66 + k]++;
        for (int i = 0; i < k; i++)
            for (int j = i + 1; j < k; j++) {
                const int a = memb[i] < memb[j] ? memb[i] : memb[j], b = memb[i] ^ memb[j] ^ a;
                bedge[beid[a * 64 + b] * 66 + k]++;
            }
        rec(cand & badj[v]);
        depth--;
    }
}

static void run_graph(const char *what, int n, const uint64_t *adj, int closed_form) {
    int32_t *rp = calloc(n + 1, sizeof *rp), *col = calloc((size_t)n * 64 + 1, sizeof *col);
    int nnz = 0;
    for (int v = 0; v < n; v++) {
        for (int u = 0; u < n; u++)
            if ((adj[v] >> u) & 1) col[nnz++] = u;
        rp[v + 1] = nnz;
    }
    const int m = nnz / 2;
    bn = n;
    badj = adj;
    bglob = calloc(66, 8);
    bvert = calloc((size_t)n * 66 + 1, 8);
    bedge = calloc((size_t)m * 66 + 1, 8);
    beid = malloc(64 * 64 * sizeof *beid);
    int e = 0;
    for (int u = 0; u < n; u++)
        for (int v = u + 1; v < n; v++) beid[u * 64 + v] = ((adj[u] >> v) & 1) ? e++ : -1;
    bglob[0] = 1;
    depth = 0;
    if (!closed_form) rec(n ? (~0ull >> (64 - n)) : 0ull);
    int omega = 0;
    if (closed_form) omega = n;
    else
        for (int k = 0; k < 66; k++)
            if (bglob[k]) omega = k;
    const int kcap = n + 3, hd = n + 2;
    const int vlo = 1, vhi = omega < 1 ? 1 : (omega > 16 ? 16 : omega), K = vhi - vlo + 1;
    const int elo = 2, ehi = omega < 2 ? 2 : (omega > 9 ? 9 : omega), EK = ehi - elo + 1;
    uint64_t *glob = calloc((size_t)kcap * 2, 8), *vc = calloc((size_t)n * K * 2 + 2, 8);
    uint64_t *ec = calloc((size_t)m * EK * 2 + 2, 8), *hist = calloc((size_t)hd * hd, 8), stats[12];
    uint8_t *govf = calloc(kcap, 1), vovf[16] = {0}, eovf[16] = {0};
    int rc = orc_count(n, rp, col, NULL, NULL, NULL, 0, 0, kcap, glob, govf, vlo, vhi, vc, vovf, elo, ehi, ec, eovf,
                       hd, hist, stats);
    CHECK(rc == 0, "%s: orc_count status %d", what, rc);
    int good = 1;
    for (int k = 0; k <= n && k < kcap; k++) {
        const u128 want = closed_form ? binom(n, k) : (k < 66 ? bglob[k] : 0);
        good &= limbs(glob + 2 * k) == want && !govf[k];
    }
    CHECK(good, "%s: global counts", what);
    CHECK((int)stats[3] == omega, "%s: omega %d, want %d", what, (int)stats[3], omega);
    /* leaf histogram: a leaf (h, p) stands for the 2^p cliques of its hold
       vertices plus any subset of its pivots, every nonempty clique once
       (Thm. scr), so the weighted leaves sum to sum_{k >= 1} C_k */
    u128 total = 0, want_total = 0;
    for (int h = 0; h < hd; h++)
        for (int p = 0; p < hd; p++)
            if (hist[h * hd + p]) total += (u128)hist[h * hd + p] << p;
    for (int k = 1; k <= n && k < kcap; k++) want_total += limbs(glob + 2 * k);
    CHECK(total == want_total && stats[8] == 0, "%s: leaf histogram", what);
    good = 1;
    for (int v = 0; v < n; v++)
        for (int k = vlo; k <= vhi; k++) {
            const u128 want = closed_form ? binom(n - 1, k - 1) : bvert[v * 66 + k];
            good &= limbs(vc + 2 * ((size_t)v * K + (k - vlo))) == want;
        }
    CHECK(good, "%s: per-vertex counts", what);
    good = 1;
    for (int x = 0; x < m; x++)
        for (int k = elo; k <= ehi; k++) {
            const u128 want = closed_form ? binom(n - 2, k - 2) : bedge[x * 66 + k];
            good &= limbs(ec + 2 * ((size_t)x * EK + (k - elo))) == want;
        }
    CHECK(good, "%s: per-edge counts", what);
    /* truncation at k_max = omega - 1, and two root subsets adding up */
    if (omega >= 2) {
        uint64_t *gt = calloc((size_t)kcap * 2, 8);
        memset(govf, 0, kcap);
        rc = orc_count(n, rp, col, NULL, NULL, NULL, 0, omega - 1, kcap, gt, govf, 0, 0, NULL, NULL, 0, 0, NULL,
                       NULL, 0, NULL, stats);
        good = rc == 0;
        for (int k = 0; k < omega; k++) good &= limbs(gt + 2 * k) == limbs(glob + 2 * k);
        CHECK(good, "%s: truncated counts", what);
        int32_t *r1 = malloc(n * sizeof *r1), *r2 = malloc(n * sizeof *r2), n1 = 0, n2 = 0;
        for (int v = 0; v < n; v++) {
            if (v % 3) r1[n1++] = v;
            else r2[n2++] = v;
        }
        uint64_t *g1 = calloc((size_t)kcap * 2, 8), *g2 = calloc((size_t)kcap * 2, 8);
        rc = orc_count(n, rp, col, NULL, NULL, r1, n1, 0, kcap, g1, govf, 0, 0, NULL, NULL, 0, 0, NULL, NULL, 0,
                       NULL, stats);
        rc |= orc_count(n, rp, col, NULL, NULL, r2, n2, 0, kcap, g2, govf, 0, 0, NULL, NULL, 0, 0, NULL, NULL, 0,
                        NULL, stats);
        good = rc == 0;
        for (int k = 1; k < kcap; k++) good &= limbs(g1 + 2 * k) + limbs(g2 + 2 * k) == limbs(glob + 2 * k);
        CHECK(good, "%s: root subsets add up", what);
        free(gt), free(r1), free(r2), free(g1), free(g2);
    }
    free(rp), free(col), free(bglob), free(bvert), free(bedge), free(beid), free(glob), free(vc), free(ec);
    free(hist), free(govf);
}

int main(void) {
    for (int a = 0; a <= 130; a++) {
        pascal[a][0] = 1;
        for (int b = 1; b <= a; b++) pascal[a][b] = pascal[a - 1][b - 1] + (b < a ? pascal[a - 1][b] : 0);
    }
    uint64_t adj[64];
    const int sizes[] = {1, 2, 5, 17, 40, 64};
    for (size_t i = 0; i < sizeof sizes / sizeof *sizes; i++) {
        const int n = sizes[i];
        for (int v = 0; v < n; v++) adj[v] = (n == 64 ? ~0ull : ((1ull << n) - 1)) & ~(1ull << v);
        char what[32];
        snprintf(what, sizeof what, "K_%d", n);
        run_graph(what, n, adj, 1);
    }
    const struct { int n; double p; } rg[] = {{30, 0.3}, {48, 0.5}, {64, 0.65}, {64, 0.05}, {20, 0.0}};
    uint64_t x = 0x9E3779B97F4A7C15ull;
    for (size_t i = 0; i < sizeof rg / sizeof *rg; i++) {
        const int n = rg[i].n;
        memset(adj, 0, sizeof adj);
        for (int v = 0; v < n; v++)
            for (int u = v + 1; u < n; u++) {
                x = x * 6364136223846793005ull + 1442695040888963407ull;
                if ((double)(x >> 11) * (1.0 / 9007199254740992.0) < rg[i].p) {
                    adj[v] |= 1ull << u;
                    adj[u] |= 1ull << v;
                }
            }
        char what[48];
        snprintf(what, sizeof what, "G(%d, %.2f)", n, rg[i].p);
        run_graph(what, n, adj, 0);
    }
    printf("oracle_check: %d checks, %d failed\n", checks, failed);
    return failed ? 1 : 0;
}
