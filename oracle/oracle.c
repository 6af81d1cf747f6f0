/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of exact clique
 * counting by pivoting (Jain & Seshadhri, "The Power of Pivoting for Exact
 * Clique Counting", WSDM 2020).  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file; the product path never
 * links, calls or imports it.  It shares no code, header or table with the
 * GPU library.
 *
 * What it computes, in the paper's order:
 *   1. A degeneracy ordering by peeling (Sec. 3, Lemma lem:degen).  The paper
 *      only says "repeatedly remove a minimum-degree vertex"; the reading
 *      used here (the "canonical peel") is: for level k = 0,1,2,..., in
 *      sub-rounds remove *all* remaining vertices whose remaining degree is
 *      <= k, until none is left at that level; the key of a vertex is
 *      (index of its sub-round, vertex id).  Edges point from the smaller key
 *      to the larger, so N+(v) = { u in N(v) : key(u) > key(v) }.
 *   2. The Succinct Clique Tree, built depth first (Sec. 4, Alg. 1; the
 *      depth-first form is the "storage cost" part of the proof of
 *      Thm. main in Sec. 5).  The root has one hold child N+(v) per vertex v.
 *      A node S != {} picks the pivot p in S maximising |N(S,p)|, makes the
 *      pivot child N(S,p), and for the non-neighbours v_1..v_l of p in S
 *      (p itself excluded) makes hold children N(S,v_i) minus {v_1..v_{i-1}}.
 *      Readings: pivot ties go to the smallest priority (default: vertex id);
 *      non-neighbours are visited in increasing priority (default: id).  Any
 *      choice gives the same counts (Thm. scr); the choices fix the tree.
 *   3. Alg. 2 (Pivoter) at each leaf, with h = |H(T)|, p = |P(T)|:
 *        global      C_{h+i}       += C(p, i)      0 <= i <= p
 *        v in H      c_{h+i}(v)    += C(p, i)      0 <= i <= p
 *        v in P      c_{h+i+1}(v)  += C(p-1, i)    0 <= i <= p-1
 *        u,v in H    c_{h+i}(e)    += C(p, i)      each unordered edge once
 *        u in P,v in H c_{h+i+1}(e) += C(p-1, i)
 *        u,v in P    c_{h+i+2}(e)  += C(p-2, i)
 *   4. Optional truncation (Sec. 5, "Counting k-cliques for a specific k"):
 *      a call whose number of hold links exceeds k_max is not made, and only
 *      counts for k <= k_max are accumulated.
 *
 * All counts are exact unsigned 128-bit integers.  A count that would reach
 * 2^128 sets its per-k overflow flag (the value is then meaningless).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------ u128 helpers */

static u128 ld128(const uint64_t *p) { return ((u128)p[1] << 64) | (u128)p[0]; }

static void st128(uint64_t *p, u128 x) {
    p[0] = (uint64_t)x;
    p[1] = (uint64_t)(x >> 64);
}

/* *acc += x with overflow flag; x_bad marks an addend that is itself >= 2^128 */
static void add128(uint64_t *acc, u128 x, int x_bad, uint8_t *flag) {
    u128 a = ld128(acc), r;
    if (x_bad || __builtin_add_overflow(a, x, &r)) {
        *flag = 1;
        r = a + x;
    }
    st128(acc, r);
}

/* -------------------------------------------------------------- the graph */

typedef struct {
    int32_t n;
    const int32_t *rp;  /* row_ptr[n+1] */
    const int32_t *col; /* sorted neighbour lists */
} graph_t;

/* is b a neighbour of a?  (binary search in the sorted row of a) */
static int adjacent(const graph_t *g, int32_t a, int32_t b) {
    int32_t lo = g->rp[a], hi = g->rp[a + 1];
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        int32_t x = g->col[mid];
        if (x == b) return 1;
        if (x < b) lo = mid + 1; else hi = mid;
    }
    return 0;
}

/* ------------------------------------------------------ 1. canonical peel */

/*
 * sub[v] <- index of the sub-round in which v is removed.  Returns the number
 * of sub-rounds; *alpha_out <- the largest level at which a vertex was
 * removed (the degeneracy).
 */
int64_t orc_peel(int32_t n, const int32_t *rp, const int32_t *col,
                 int32_t *sub, int32_t *alpha_out) {
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    uint8_t *alive = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    uint8_t *take = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    int32_t *alive_list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t nalive = n;
    for (int32_t v = 0; v < n; v++) {
        deg[v] = rp[v + 1] - rp[v];
        alive[v] = 1;
        take[v] = 0;
        alive_list[v] = v;
    }
    int64_t r = 0;
    int32_t k = 0, alpha = 0;
    while (nalive > 0) {
        /* the frontier of this sub-round: every remaining vertex of degree <= k */
        int32_t cnt = 0;
        for (int32_t i = 0; i < nalive; i++) {
            int32_t v = alive_list[i];
            if (deg[v] <= k) { take[v] = 1; cnt++; }
        }
        if (cnt == 0) { k++; continue; } /* nothing left at this level */
        if (k > alpha) alpha = k;
        for (int32_t i = 0; i < nalive; i++) {
            int32_t v = alive_list[i];
            if (take[v]) { alive[v] = 0; sub[v] = (int32_t)r; }
        }
        for (int32_t i = 0; i < nalive; i++) {
            int32_t v = alive_list[i];
            if (!take[v]) continue;
            for (int32_t e = rp[v]; e < rp[v + 1]; e++)
                if (alive[col[e]]) deg[col[e]]--;
        }
        int32_t w = 0;
        for (int32_t i = 0; i < nalive; i++) {
            int32_t v = alive_list[i];
            if (take[v]) take[v] = 0; else alive_list[w++] = v;
        }
        nalive = w;
        r++;
    }
    if (alpha_out) *alpha_out = alpha;
    free(deg); free(alive); free(take); free(alive_list);
    return r;
}

/* ----------------------------------------------------- 2+3. SCT and Alg. 2 */

typedef struct {
    graph_t g;
    const int32_t *key;  /* orientation key part 1 (sub-round); ties by id */
    const int32_t *prio; /* tie-break priority (NULL: vertex id) */
    int32_t kmax;        /* 0: no truncation */

    int32_t bn;          /* binomial table is bn x bn */
    u128 *binom;
    uint8_t *bbad;       /* C(a,b) >= 2^128 */

    int32_t kcap;        /* global counts 0..kcap-1 */
    uint64_t *glob;      /* [kcap][2] */
    uint8_t *govf;

    int32_t vlo, vhi;    /* per-vertex range, vc = [n][K][2] */
    uint64_t *vc;
    uint8_t *vovf;

    int32_t elo, ehi;    /* per-edge range, ec = [m][K][2] */
    uint64_t *ec;
    uint8_t *eovf;
    int64_t *eoff;       /* eoff[v] = number of edges (a,b), a<b, with a<v */
    int32_t *efirst;     /* efirst[v] = position of the first neighbour > v in row v */

    int32_t hd;          /* leaf histogram hist[h][p], hd x hd */
    uint64_t *hist;

    uint64_t nodes, leaves, work_sw, hist_out;
    uint64_t work_child; /* sum over internal nodes of (children) * ceil(|S|/64) */
    uint64_t leaf_hp;    /* sum over leaves of h + p */
    uint64_t leaf_pairs; /* sum over leaves of C(h + p, 2) */
    int32_t maxdepth, omega, need_kcap;
    int32_t *H, *P;      /* current path (hold / pivot vertices) */
    int32_t *arena;      /* one buffer of alpha+1 ints per depth */
    int32_t astride;
    int32_t err;
} orc_t;

static int32_t prio_of(const orc_t *o, int32_t v) { return o->prio ? o->prio[v] : v; }

/* key(a) < key(b): orientation a -> b */
static int key_less(const orc_t *o, int32_t a, int32_t b) {
    if (o->key[a] != o->key[b]) return o->key[a] < o->key[b];
    return a < b;
}

static void binom_of(const orc_t *o, int32_t a, int32_t b, u128 *val, int *bad) {
    if (b < 0 || a < 0 || b > a) { *val = 0; *bad = 0; return; }
    *val = o->binom[(size_t)a * o->bn + b];
    *bad = o->bbad[(size_t)a * o->bn + b];
}

static int64_t edge_id(const orc_t *o, int32_t a, int32_t b) {
    if (a > b) { int32_t t = a; a = b; b = t; }
    int32_t lo = o->g.rp[a], hi = o->g.rp[a + 1];
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (o->g.col[mid] < b) lo = mid + 1; else hi = mid;
    }
    return o->eoff[a] + (lo - o->efirst[a]);
}

/* add C(pp, i) to c_{base+i}(e) for 0 <= i <= pp */
static void edge_add(orc_t *o, int32_t a, int32_t b, int32_t base, int32_t pp) {
    int32_t K = o->ehi - o->elo + 1;
    int64_t id = edge_id(o, a, b);
    for (int32_t i = 0; i <= pp; i++) {
        int32_t k = base + i;
        if (k < o->elo || k > o->ehi) continue;
        if (o->kmax && k > o->kmax) continue;
        u128 c; int bad;
        binom_of(o, pp, i, &c, &bad);
        add128(o->ec + ((size_t)id * K + (k - o->elo)) * 2, c, bad, &o->eovf[k - o->elo]);
    }
}

static void vertex_add(orc_t *o, int32_t v, int32_t base, int32_t pp) {
    int32_t K = o->vhi - o->vlo + 1;
    for (int32_t i = 0; i <= pp; i++) {
        int32_t k = base + i;
        if (k < o->vlo || k > o->vhi) continue;
        if (o->kmax && k > o->kmax) continue;
        u128 c; int bad;
        binom_of(o, pp, i, &c, &bad);
        add128(o->vc + ((size_t)v * K + (k - o->vlo)) * 2, c, bad, &o->vovf[k - o->vlo]);
    }
}

/* Alg. 2 applied to one root-to-leaf path */
static void leaf(orc_t *o, int32_t h, int32_t p) {
    o->leaves++;
    o->leaf_hp += (uint64_t)(h + p);
    o->leaf_pairs += (uint64_t)(h + p) * (uint64_t)(h + p - 1) / 2;
    if (h + p > o->omega) o->omega = h + p;
    if (o->hist && h < o->hd && p < o->hd) o->hist[(size_t)h * o->hd + p]++;
    else if (o->hist) o->hist_out++;
    if (h + p + 1 > o->need_kcap) o->need_kcap = h + p + 1;
    if (h + p >= o->kcap) { o->err = -7; return; }
    /* global counts */
    for (int32_t i = 0; i <= p; i++) {
        int32_t k = h + i;
        if (o->kmax && k > o->kmax) break;
        u128 c; int bad;
        binom_of(o, p, i, &c, &bad);
        add128(o->glob + (size_t)k * 2, c, bad, &o->govf[k]);
    }
    /* per-vertex counts */
    if (o->vc) {
        for (int32_t j = 0; j < h; j++) vertex_add(o, o->H[j], h, p);
        for (int32_t j = 0; j < p; j++) vertex_add(o, o->P[j], h + 1, p - 1);
    }
    /* per-edge counts, each unordered pair once */
    if (o->ec) {
        for (int32_t a = 0; a < h; a++)
            for (int32_t b = a + 1; b < h; b++) edge_add(o, o->H[a], o->H[b], h, p);
        for (int32_t a = 0; a < p; a++)
            for (int32_t b = 0; b < h; b++) edge_add(o, o->P[a], o->H[b], h + 1, p - 1);
        for (int32_t a = 0; a < p; a++)
            for (int32_t b = a + 1; b < p; b++) edge_add(o, o->P[a], o->P[b], h + 2, p - 2);
    }
}

/*
 * One SCT node labelled S (s vertices, any order), reached by a path with
 * h hold vertices H[0..h-1] and p pivot vertices P[0..p-1].
 */
static void rec(orc_t *o, const int32_t *S, int32_t s, int32_t h, int32_t p, int32_t depth) {
    o->nodes++;
    o->work_sw += (uint64_t)s * (uint64_t)((s + 63) / 64);
    if (depth > o->maxdepth) o->maxdepth = depth;
    if (o->err) return;
    if (s == 0) { leaf(o, h, p); return; }

    /* pivot: the vertex of S with the most neighbours inside S */
    int32_t best = -1, bestc = -1;
    for (int32_t i = 0; i < s; i++) {
        int32_t c = 0;
        for (int32_t j = 0; j < s; j++)
            if (j != i && adjacent(&o->g, S[i], S[j])) c++;
        if (c > bestc || (c == bestc && prio_of(o, S[i]) < prio_of(o, S[best]))) {
            best = i;
            bestc = c;
        }
    }
    int32_t piv = S[best];
    int32_t *child = o->arena + (size_t)(depth + 1) * o->astride;

    /* pivot child N(S, piv), link (piv, pivot) */
    int32_t cs = 0;
    for (int32_t j = 0; j < s; j++)
        if (adjacent(&o->g, piv, S[j])) child[cs++] = S[j];
    o->P[p] = piv;
    o->work_child += (uint64_t)((s + 63) / 64); /* the pivot child */
    rec(o, child, cs, h, p + 1, depth + 1);

    /* hold children: the non-neighbours v_1, v_2, ... of piv in S (piv itself
       excluded), visited in increasing priority; child i is N(S, v_i) minus
       {v_1, ..., v_{i-1}}, link (v_i, hold) */
    int first = 1;
    int32_t last = 0;
    for (;;) {
        int32_t v = -1;
        for (int32_t j = 0; j < s; j++) {
            int32_t x = S[j];
            if (x == piv || adjacent(&o->g, piv, x)) continue;
            if (!first && prio_of(o, x) <= last) continue;
            if (v < 0 || prio_of(o, x) < prio_of(o, v)) v = x;
        }
        if (v < 0) break;
        if (o->kmax && h + 1 > o->kmax) break; /* more than kmax hold links */
        cs = 0;
        for (int32_t j = 0; j < s; j++) {
            int32_t x = S[j];
            if (!adjacent(&o->g, v, x)) continue;
            /* x is an earlier non-neighbour of piv: excluded */
            if (x != piv && !adjacent(&o->g, piv, x) && prio_of(o, x) < prio_of(o, v)) continue;
            child[cs++] = x;
        }
        o->H[h] = v;
        o->work_child += (uint64_t)((s + 63) / 64); /* a hold child */
        rec(o, child, cs, h + 1, p, depth + 1);
        last = prio_of(o, v);
        first = 0;
    }
}

/*
 * Count cliques of the graph (row_ptr, col: symmetric, sorted, simple).
 *
 * key_in  : orientation key per vertex (edge a->b iff (key[a],a) < (key[b],b));
 *           NULL: the canonical peel computed here.
 * prio    : distinct tie-break priorities (NULL: vertex ids).
 * roots   : process only these root children of the SCT (NULL: all vertices).
 *           The result for a root subset counts the cliques whose smallest-key
 *           vertex is in the subset.
 * kmax    : 0, or the truncation bound on hold links.
 * glob    : [kcap][2] u64 (lo, hi) global counts C_0..C_{kcap-1}; govf[kcap].
 * vc      : NULL or [n][vhi-vlo+1][2] per-vertex counts; vovf[K].
 * ec      : NULL or [m][ehi-elo+1][2] per-edge counts, edge id = rank of (u,v),
 *           u<v, in lexicographic order; eovf[K].
 * hist    : NULL or [hd][hd] leaf histogram by (h, p).
 * stats   : [12] nodes, leaves, alpha, omega, max depth, sum |S|*ceil(|S|/64),
 *           sub-rounds of the peel (0 if key_in given), kcap needed,
 *           leaves outside the histogram, then the work counters of the
 *           roofline model: sum over internal nodes of (children made) *
 *           ceil(|S|/64) (one word operation per child and word of S),
 *           sum over leaves of h + p, sum over leaves of C(h + p, 2).
 * Returns 0, -7 if kcap is too small (stats[7] says what is needed), -3 on
 * allocation failure.
 */
int32_t orc_count(int32_t n, const int32_t *rp, const int32_t *col,
                  const int32_t *key_in, const int32_t *prio,
                  const int32_t *roots, int32_t nroots, int32_t kmax,
                  int32_t kcap, uint64_t *glob, uint8_t *govf,
                  int32_t vlo, int32_t vhi, uint64_t *vc, uint8_t *vovf,
                  int32_t elo, int32_t ehi, uint64_t *ec, uint8_t *eovf,
                  int32_t hd, uint64_t *hist, uint64_t *stats) {
    orc_t o;
    memset(&o, 0, sizeof(o));
    o.g.n = n;
    o.g.rp = rp;
    o.g.col = col;
    o.prio = prio;
    o.kmax = kmax;
    o.kcap = kcap;
    o.glob = glob;
    o.govf = govf;
    o.vlo = vlo; o.vhi = vhi; o.vc = vc; o.vovf = vovf;
    o.elo = elo; o.ehi = ehi; o.ec = ec; o.eovf = eovf;
    o.hd = hd; o.hist = hist;

    int32_t *key_own = NULL;
    int64_t subrounds = 0;
    if (!key_in) {
        key_own = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        if (!key_own) return -3;
        int32_t a;
        subrounds = orc_peel(n, rp, col, key_own, &a);
        o.key = key_own;
    } else {
        o.key = key_in;
    }

    /* out-degrees under the orientation */
    int32_t alpha = 0;
    for (int32_t v = 0; v < n; v++) {
        int32_t d = 0;
        for (int32_t e = rp[v]; e < rp[v + 1]; e++)
            if (key_less(&o, v, col[e])) d++;
        if (d > alpha) alpha = d;
    }

    /* exact binomial table (Pascal's rule), with a flag for values >= 2^128 */
    o.bn = alpha + 3;
    o.binom = (u128 *)calloc((size_t)o.bn * o.bn, sizeof(u128));
    o.bbad = (uint8_t *)calloc((size_t)o.bn * o.bn, 1);
    o.astride = alpha + 1;
    o.arena = (int32_t *)malloc(sizeof(int32_t) * (size_t)(alpha + 4) * (size_t)o.astride);
    o.H = (int32_t *)malloc(sizeof(int32_t) * (size_t)(alpha + 3));
    o.P = (int32_t *)malloc(sizeof(int32_t) * (size_t)(alpha + 3));
    if (!o.binom || !o.bbad || !o.arena || !o.H || !o.P) {
        free(o.binom); free(o.bbad); free(o.arena); free(o.H); free(o.P); free(key_own);
        return -3;
    }
    for (int32_t a = 0; a < o.bn; a++) {
        o.binom[(size_t)a * o.bn + 0] = 1;
        for (int32_t b = 1; b <= a; b++) {
            u128 x = o.binom[(size_t)(a - 1) * o.bn + b - 1];
            u128 y = (b <= a - 1) ? o.binom[(size_t)(a - 1) * o.bn + b] : 0;
            int bad = o.bbad[(size_t)(a - 1) * o.bn + b - 1] ||
                      (b <= a - 1 && o.bbad[(size_t)(a - 1) * o.bn + b]);
            u128 r;
            if (__builtin_add_overflow(x, y, &r)) bad = 1;
            o.binom[(size_t)a * o.bn + b] = r;
            o.bbad[(size_t)a * o.bn + b] = (uint8_t)bad;
        }
    }

    /* edge ids */
    if (ec) {
        o.eoff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
        o.efirst = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        int64_t acc = 0;
        for (int32_t v = 0; v < n; v++) {
            int32_t e = rp[v];
            while (e < rp[v + 1] && col[e] < v) e++;
            o.efirst[v] = e;
            o.eoff[v] = acc;
            acc += rp[v + 1] - e;
        }
        o.eoff[n] = acc;
    }

    if (!roots && kcap > 0) {
        st128(glob, 1); /* C_0 = 1: the empty clique */
    }

    /* the root has one hold child per vertex v, labelled N+(v) (no pivot) */
    int32_t *S0 = o.arena; /* depth 0 buffer */
    int32_t count = roots ? nroots : n;
    for (int32_t t = 0; t < count && !o.err; t++) {
        int32_t v = roots ? roots[t] : t;
        int32_t s = 0;
        for (int32_t e = rp[v]; e < rp[v + 1]; e++)
            if (key_less(&o, v, col[e])) S0[s++] = col[e];
        o.H[0] = v;
        rec(&o, S0, s, 1, 0, 0);
    }

    if (stats) {
        stats[0] = o.nodes;
        stats[1] = o.leaves;
        stats[2] = (uint64_t)alpha;
        stats[3] = (uint64_t)o.omega;
        stats[4] = (uint64_t)o.maxdepth;
        stats[5] = o.work_sw;
        stats[6] = (uint64_t)subrounds;
        stats[7] = (uint64_t)o.need_kcap;
        stats[8] = o.hist_out;
        stats[9] = o.work_child;
        stats[10] = o.leaf_hp;
        stats[11] = o.leaf_pairs;
    }
    free(o.binom); free(o.bbad); free(o.arena); free(o.H); free(o.P);
    free(o.eoff); free(o.efirst); free(key_own);
    return o.err;
}
