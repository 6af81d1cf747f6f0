/*
 * pivoter.h -- C ABI of the MI355X exact clique counter.
 *
 * The library counts k-cliques exactly, for every k at once, by building the
 * Succinct Clique Tree (SCT) of a graph on the GPU and reading the counts off
 * its leaves (Jain & Seshadhri, "The Power of Pivoting for Exact Clique
 * Counting", WSDM 2020):
 *
 *   - degeneracy orientation (Sec. 3, Lemma lem:degen; Alg. 1 first step),
 *   - SCT built depth first by pivoting on every vertex's out-neighbourhood
 *     (Sec. 4, Alg. 1; depth-first form from the proof of Thm. main),
 *   - counts from the leaves (Sec. 5, Alg. 2): a leaf whose root-to-leaf
 *     path has h hold vertices and p pivot vertices represents C(p, i)
 *     cliques of size h + i (Thm. scr), which gives global, per-vertex and
 *     per-edge counts,
 *   - optional truncation at k_max hold vertices (Sec. 5, "Counting
 *     k-cliques for a specific k").
 *
 * Conventions (all entry points):
 *   - Plain C types only; pointers are host pointers unless the name or the
 *     comment says "device".  Device pointers are HIP device addresses on the
 *     context's device.
 *   - Vertex ids are int32 in [0, n).  A graph is simple and undirected; its
 *     CSR lists every edge in both directions with sorted rows.
 *   - Counts are exact unsigned 128-bit integers, stored as pv_u128
 *     {lo, hi} (little-endian limbs).  A count that reaches 2^128 is not
 *     representable: its overflow bit is set and its value is meaningless.
 *     pv_count_global_wide returns global counts in any number of limbs.
 *   - Every entry point returns a pv_status; nothing throws across the ABI.
 *     On error the outputs are unspecified and the handles stay valid.
 *   - Work is issued on the context's HIP stream.  Entry points that return
 *     results in host memory synchronise that stream before returning;
 *     pv_count writes device outputs and synchronises too (it returns host
 *     counters).  A context is not thread-safe; use one per host thread.
 */
#ifndef PIVOTER_H
#define PIVOTER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    uint64_t lo, hi;
} pv_u128;

typedef int32_t pv_status;

#define PV_OK 0
#define PV_EINVAL -1       /* bad argument (null pointer, bad range, ...) */
#define PV_ENOTSIMPLE -2   /* CSR not simple/symmetric/sorted (loop, duplicate, missing reverse edge) */
#define PV_ENOMEM -3       /* host or device allocation failed */
#define PV_EOVERFLOW -4    /* some requested count is >= 2^128; see overflow bits */
#define PV_EDEVICE -5      /* HIP runtime error */
#define PV_ETOOBIG -6      /* n or 2m does not fit int32, or the degeneracy exceeds the supported bound */
#define PV_EBUFSIZE -7     /* output buffer too small; required size reported */
#define PV_ECANCELLED -8   /* request cancelled */
#define PV_EAGAIN -9       /* not admitted now (memory budget); retry later */
#define PV_ETIMEDOUT -10   /* the call ran past the context's timeout and was stopped */

/* local count kinds */
#define PV_NONE 0
#define PV_VERTEX 1
#define PV_EDGE 2

/* flags of pv_graph_load_csr* (the paper counts cliques of a simple
   undirected graph and drops edge directions and repeats, Sec. 6's input
   preparation; the repair flags do that here) */
#define PV_TRUST_INPUT 1u  /* skip the simple/symmetric/sorted validation */
#define PV_DEDUP 2u        /* repair: sort every row, drop repeated entries and self loops */
#define PV_SYMMETRIZE 4u   /* repair: add the reverse of every entry (then as PV_DEDUP) */

/* largest supported degeneracy (out-degree bound of the orientation) */
#define PV_MAX_ALPHA 4096
/* one tree walk keeps local counts for at most this many consecutive k
   (pv_count_local covers wider ranges window by window) */
#define PV_MAX_LOCAL_K 16

typedef struct pv_ctx pv_ctx;
typedef struct pv_graph pv_graph;

/* Work counters of the last count call on a graph. */
typedef struct {
    uint64_t nodes;        /* SCT nodes below the root V that were visited */
    uint64_t leaves;       /* SCT leaves (root-to-leaf paths) */
    uint64_t items;        /* subproblems handed between GPU stages */
    uint64_t work;         /* pivot work: sum over nodes of |S| * ceil(|S|/64) */
    int32_t alpha;         /* degeneracy = largest out-degree */
    int32_t omega;         /* largest clique size (0 for the empty graph) */
    int32_t subrounds;     /* sub-rounds of the degeneracy peel */
    int32_t truncated;     /* 1 if the tree was cut at k_max hold vertices */
    int32_t levels;        /* launches of the SCT level kernel */
    float ms_peel;         /* device time of the peel kernel          \ HIP events on */
    float ms_orient;       /* device time of the N+(v) construction    | the context */
    float ms_levels;       /* summed device time of the level kernels  | stream, only */
    float ms_finalize;     /* device time of the u128 finalize kernel / with timing on */
    /* the level kernel per unit kind: [0] multi-word nodes and heavy roots,
       [1] compact node and frame items, [2] light roots */
    uint32_t launches_kind[3];  /* launches */
    float ms_kind[3];           /* summed device time (timing on) */
    uint64_t work_kind[3];      /* pivot work done by that kind's launches */
    int32_t kernel_kl;          /* the level kernel's k-slots (0: global counts only) */
    int32_t kernel_lk;          /* its local-count kind: 0 per vertex (u128 visit sums),
                                   1 per edge, 2 per vertex (u64 visit sums) */
    int32_t attempts;           /* walks of the tree: 1, plus one rerun per work-buffer overflow */
    /* algorithmic work of the walk (the terms of its roofline model) */
    uint64_t child_work;        /* sum over internal nodes of children * ceil(|S|/64): the word
                                   operations that form the children's vertex sets */
    uint64_t leaf_hp;           /* sum over leaves of h + p: per-vertex additions per value of k */
    uint64_t leaf_pp;           /* sum over leaves of p + 1: global additions (one per k <= p + h) */
    int32_t heavy_chunks;       /* chunks the heavy roots were walked in (their level buffers are
                                   halved until one chunk's fit the device or the budget) */
} pv_stats;

/* Human-readable name of a status code (static string). */
const char *pv_strerror(pv_status s);

/*
 * Configuration of a context (pv_init).  Zero fields take the defaults.
 *   stream      hipStream_t to issue work on (NULL: the legacy default stream).
 *   hbm_budget  bytes of device memory the context may hold at once: its
 *               workspaces and the graphs loaded through it.  An allocation
 *               that would pass it fails with PV_ENOMEM, as if the device
 *               were that small (0: no limit besides the device).
 *   tune_cache  path of the tuning cache, a JSON file written by pv_autotune
 *               and read by pv_init (NULL: none).  A graph whose key (device
 *               name and out-degree histogram, see pv_autotune) is in the
 *               cache is walked with the cached settings.
 *   dfs_max, dfs_budget, lane_max: the tuning settings below (0: default;
 *               lane_max -1 turns the lane tier off).
 *   timeout_ms  watchdog of every count call on the context: a walk still
 *               running after this many milliseconds is stopped (its waves
 *               take no further units) and the call returns PV_ETIMEDOUT,
 *               leaving the context usable (0: none).
 */
typedef struct {
    void *stream;
    int64_t hbm_budget;
    const char *tune_cache;
    int32_t dfs_max;
    int32_t dfs_budget;
    int32_t lane_max;
    int32_t timeout_ms;
} pv_config;

/*
 * Create a context on HIP device `device` with configuration `cfg` (NULL:
 * all defaults).  The context owns the binomial table and per-device
 * workspaces; it is released by pv_fini.
 */
pv_status pv_init(int32_t device, const pv_config *cfg, pv_ctx **out);
void pv_fini(pv_ctx *ctx);

/*
 * Cancel the count call running on the context now, from any host thread:
 * its waves take no further units, and the call returns PV_ECANCELLED once
 * the units in hand are done (a unit walks at most the depth-first budget
 * of nodes).  The context stays usable; no effect when no call runs.
 * Results are not partial: a cancelled call's outputs are undefined and the
 * call is simply run again.  The flag is raised on a HIP stream of the
 * context's own, created by the first pv_cancel of a context without a
 * timeout (PV_EDEVICE if that fails); the calling thread's current device is
 * left as it was.
 */
pv_status pv_cancel(pv_ctx *ctx);

/* Device bytes the context holds now (workspaces and its graphs). */
pv_status pv_memory(const pv_ctx *ctx, int64_t *held_bytes);

/*
 * Measured peaks of the context's device, the denominators of the walk's
 * roofline model (no passage of the method defines them: they are the
 * device's own rates).  Each figure is the best of five timed runs on the
 * context's stream after one untimed run:
 *   hbm_copy_gbs  stream copy of copy_bytes (0: 1 GiB) between two device
 *                 buffers, counting the bytes read plus the bytes written;
 *   hbm_read_gbs  stream read of copy_bytes;
 *   lds_read_gbs  64-bit LDS reads, conflict free, summed over all CUs;
 *   valu_gops     32-bit VALU lane operations per second (XOR then
 *                 popcount-accumulate, the pivot search's instructions).
 * ms_* are the best kernel times.  Allocates 2 * copy_bytes of device
 * memory (charged to the context's budget: PV_ENOMEM past it) and frees it
 * before returning; synchronises the stream.
 */
typedef struct {
    double hbm_copy_gbs;
    double hbm_read_gbs;
    double lds_read_gbs;
    double valu_gops;
    float ms_copy, ms_read, ms_lds, ms_valu;
} pv_peaks;
pv_status pv_measure_peaks(pv_ctx *ctx, int64_t copy_bytes, pv_peaks *out);

/*
 * Environment variables read by pv_init besides the tuning defaults below;
 * none changes a result, they choose how the work is split:
 *   PV_HU_BUDGET    bytes of device memory for the gathered neighbourhoods
 *                   of heavy roots (|N+(v)| > 64) per pass over them; the
 *                   roots are taken in as many chunks as that needs
 *                   (default 2^30, at most a quarter of hbm_budget).
 *   PV_PREFIX_ROWS  per-vertex counts: rows of N+(root) summed per on-chip
 *                   pass when what the universes owe the vertices above them
 *                   is added up per heavy root (default: as many as fit).
 *   PV_DEBUG        per-level buffer demands and times on stderr.
 *   PV_PACK         local counts: 0 sends every addition straight to the
 *                   u128 output; by default, when no count can reach 2^62
 *                   (per edge n * C(alpha, k - 2), per vertex
 *                   (max degree + 1) * C(alpha, k - 1), for every k asked
 *                   for; per vertex only with 64-bit visit sums), two values
 *                   of k share one 64-bit atomic in 32-bit halves and the
 *                   carries are counted beside them.
 *   PV_PACK_BIAS    local counts, packed: the halves' starting value
 *                   (default 0; a value near 2^32 makes them wrap after a
 *                   few additions, which tests use).
 *   PV_RECORD       a file path: every count call on the context appends
 *                   one JSON line to it (the call, the graph's n and m,
 *                   alpha, omega, k_max, the local range, the walk's
 *                   counters from pv_stats, the device times and the
 *                   returned status).  Appends are serialised within the
 *                   process; a file that cannot be opened is skipped.
 */

/* Change the stream later work is issued on (hipStream_t, may be NULL). */
pv_status pv_set_stream(pv_ctx *ctx, void *stream);

/*
 * Tuning: subtrees whose node set has at most dfs_max vertices (1..64) are
 * walked depth first by one wavefront; larger nodes are split so that their
 * hold children are spread over the GPU.  Any value gives the same counts.
 * Default 64 (environment variable PV_DFS_MAX overrides it at pv_init).
 */
pv_status pv_set_dfs_max(pv_ctx *ctx, int32_t dfs_max);

/*
 * Record HIP events around the peel, orientation, level and finalize
 * kernels of later calls (on = 1) and report their device times in
 * pv_stats.  Off by default.
 */
pv_status pv_set_timing(pv_ctx *ctx, int32_t on);

/*
 * Tuning: a wavefront walks at most this many SCT nodes depth first before
 * it hands the rest of its subtree (the pending node and the pending hold
 * children on its stack) to other wavefronts.  Any value in [16, 2^20]
 * gives the same counts.  0 (the default) picks it per tree level: 4096
 * for global counts alone; with local counts 8192, or 2048 on a level with
 * fewer than 16 units per wavefront.  PV_DFS_BUDGET overrides the default
 * at pv_init.
 */
pv_status pv_set_dfs_budget(pv_ctx *ctx, int32_t nodes);

/*
 * Tuning: subtrees whose node set has at most lane_max vertices (0..8) are
 * walked one per lane, up to 64 at once per wavefront, instead of one node
 * at a time by the whole wavefront.  0 turns this off.  Any value gives the
 * same counts and tree.  Default 8 (PV_LANE_MAX overrides it at pv_init).
 * Used for global counts, and for per-vertex counts of at most 8 values of
 * k whose per-visit sums fit 64 bits.
 */
pv_status pv_set_lane_max(pv_ctx *ctx, int32_t lane_max);

/*
 * Autotuning of how the walk is split (the tile widths of the batched
 * persistent walk: which subtrees go one per lane, which one per
 * wavefront, and how many nodes a wavefront walks before it hands work
 * back to the queue).  No setting changes a count, a tree or a statistic
 * other than timings (Thm. scr: the tree depends only on the pivot and
 * order rules, which stay fixed).
 *
 * pv_autotune times pv_count on g (global counts for all k, plus the given
 * local counts, local_out being a DEVICE buffer as pv_count's) under
 * candidate settings, one setting at a time from the current best
 * (lane_max in {0,4,6,8}; dfs_budget in {auto,1024,...,16384}; dfs_max in
 * {32,48,64}), each the best of `reps` runs (>= 1).  The winner is kept
 * for the graph's key, which is the device (architecture and CU count),
 * the kind of count, and the out-degree histogram in powers of two with
 * each count rounded to its power of two; later pv_count / pv_count_batch
 * calls on this context use it for graphs with the same key, and with a
 * tune_cache path (pv_config) it is also written to that JSON file, which
 * later contexts read.
 */
typedef struct {
    int32_t dfs_max;      /* chosen settings */
    int32_t dfs_budget;   /* 0: chosen per tree level */
    int32_t lane_max;     /* 0: lane tier off */
    float ms_best;        /* best time of one pv_count with them */
    float ms_default;     /* best time with the context's settings before tuning */
    int32_t trials;       /* settings timed */
} pv_tune;

pv_status pv_autotune(pv_graph *g, int32_t local_kind, int32_t k_lo, int32_t k_hi, pv_u128 *local_out,
                      int32_t reps, pv_tune *out);

/* The key under which g's tuned settings are kept (static storage of this
   host thread, valid until the next call on it). */
const char *pv_tune_key(pv_graph *g, int32_t local_kind, int32_t k_lo, int32_t k_hi);

/* Text of the last HIP error seen by this host thread (static storage). */
const char *pv_last_error(void);

/*
 * Load a graph from a host CSR: row_ptr[n+1], col[row_ptr[n]], rows sorted,
 * every undirected edge listed in both directions, no self loops or
 * duplicates (problem statement, Sec. 1.1: a simple undirected graph).
 * The inputs are copied; the caller keeps ownership.  Unless
 * PV_TRUST_INPUT is set the CSR is validated (PV_ENOTSIMPLE otherwise).
 * PV_DEDUP and PV_SYMMETRIZE repair the copy first (on the host); a column
 * id outside [0, n) cannot be repaired and gives PV_ENOTSIMPLE.  Isolated
 * vertices are allowed.  The graph handle owns its device memory.
 */
pv_status pv_graph_load_csr(pv_ctx *ctx, int32_t n, const int32_t *row_ptr,
                            const int32_t *col, uint32_t flags, pv_graph **out);

/* Same, from a CSR already in device memory (device pointers of the
   context's device, copied; problem statement, Sec. 1.1).  nnz = row_ptr[n].
   With a repair flag the CSR takes a round trip through host memory. */
pv_status pv_graph_load_csr_device(pv_ctx *ctx, int32_t n, int64_t nnz,
                                   const int32_t *d_row_ptr, const int32_t *d_col,
                                   uint32_t flags, pv_graph **out);

/* Release a graph and its device memory.  PV_EAGAIN (nothing released) while
   a count on another host thread uses it. */
pv_status pv_graph_free(pv_graph *g);

/* n and m (undirected edges) of a loaded graph. */
pv_status pv_graph_size(const pv_graph *g, int32_t *n, int64_t *m);

/*
 * Degeneracy orientation (Sec. 3, Lemma lem:degen).  Peel level k = 0,1,...:
 * in sub-rounds remove every remaining vertex of remaining degree <= k; a
 * vertex's key is (its sub-round, its id) and every edge points from the
 * smaller key to the larger.  Out-degrees are then at most the degeneracy
 * alpha (returned if alpha_out != NULL).  Always recomputed (idempotent);
 * the count calls orient first if it has not been done.
 */
pv_status pv_graph_orient(pv_graph *g, int32_t *alpha_out);

/* Copy the peel sub-round of every vertex (int32[n], host): the key of the
   degeneracy order of Sec. 3, Lemma lem:degen (ties by vertex id). */
pv_status pv_graph_export_order(pv_graph *g, int32_t *sub_host);

/*
 * Global counts C_k (problem statement, Sec. 1.1; read off by Alg. 2's
 * global step).  counts[k] = C_k for 0 <= k < cap, with counts[0] = 1 (the
 * empty clique), counts[1] = n, counts[2] = m, and zeros above omega.
 * k_max <= 0: all k; otherwise the tree is truncated at k_max hold vertices
 * (Sec. 5) and counts above k_max are zero.
 * overflow_bits (may be NULL): uint64[(cap+63)/64], bit k set if C_k >= 2^128
 * (PV_EOVERFLOW is returned then).  PV_EBUFSIZE if cap <= min(omega, k_max)
 * (omega_out still set).  stats may be NULL.
 */
pv_status pv_count_global(pv_graph *g, int32_t k_max, pv_u128 *counts, int32_t cap,
                          int32_t *omega_out, uint64_t *overflow_bits, pv_stats *stats);

/*
 * Global counts C_k wider than 128 bits (Sec. 5's read-off, C_k = the sum
 * over SCT leaves (h, p) of C(p, k - h), done in multi-limb integers; the
 * paper's graphs with a clique number above about 130 need it).  Same tree
 * and same k_max rule as pv_count_global.
 *   counts: host memory, [cap][limbs] uint64, little-endian limbs:
 *           counts[k * limbs + i] holds bits 64i..64i+63 of C_k.
 *   limbs >= 1.  overflow_bits (may be NULL): uint64[(cap+63)/64], bit k set
 *   if C_k >= 2^(64 limbs); those limbs then hold C_k mod 2^(64 limbs) and
 *   PV_EOVERFLOW is returned.  PV_EBUFSIZE if cap <= min(omega, k_max).
 *   PV_ENOMEM if the exact binomial table for the clique number (omega + 1
 *   rows of omega + 1 entries of ceil((omega + 1) / 64) limbs) would pass
 *   2 GiB, that is omega above about 1600.  stats may be NULL.
 */
pv_status pv_count_global_wide(pv_graph *g, int32_t k_max, uint64_t *counts, int32_t cap, int32_t limbs,
                               int32_t *omega_out, uint64_t *overflow_bits, pv_stats *stats);

/*
 * Frequency distribution of local counts (Sec. 6, demonstrations: f_k(b),
 * the number of vertices that take part in exactly b k-cliques; on a
 * per-edge table, the number of edges).  local: DEVICE memory, a [rows][K]
 * pv_u128 table such as pv_count writes (column col holds k = k_lo + col).
 * values / freq: host memory of cap entries; on success values[0..D) are
 * the D distinct counts of the column in increasing order (0 included when
 * present) and freq[i] the number of rows holding values[i], so the freq
 * sum to rows.  *ndistinct = D (set also when PV_EBUFSIZE: cap < D; nothing
 * else is written then).  rows < 2^31 - 1; the context's stream is used
 * and the call returns when the results are in host memory.
 */
pv_status pv_local_frequency(pv_ctx *ctx, const pv_u128 *local, int64_t rows, int32_t K, int32_t col,
                             pv_u128 *values, uint64_t *freq, int64_t cap, int64_t *ndistinct);

/*
 * pv_local_frequency without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid it): the same inputs, outputs and results,
 * with every intermediate in a fixed scratch array of the library's (about
 * 52 MiB per device, held from the first pv_init on that device until the
 * process ends).  rows is at most PV_FREQ_STATIC_ROWS (PV_ETOOBIG beyond,
 * with nothing launched).  The call makes no device or host allocation of
 * its own.  All calls on one device share that array, so calls that overlap
 * on one device (several host threads or streams) race: the caller
 * serialises them.
 */
#define PV_FREQ_STATIC_ROWS (1 << 20)
pv_status pv_local_frequency_static(pv_ctx *ctx, const pv_u128 *local, int64_t rows, int32_t K, int32_t col,
                                    pv_u128 *values, uint64_t *freq, int64_t cap, int64_t *ndistinct);

/*
 * Local counts for k_lo <= k <= k_hi (1 <= k_lo <= k_hi <= PV_MAX_ALPHA + 1),
 * Alg. 2 per-vertex and per-edge steps.  The binomials C(alpha, b) for
 * b < k_hi must fit 64 bits (PV_ETOOBIG otherwise; every k when alpha <= 67).
 *   kind PV_VERTEX: out[v*K + (k-k_lo)] = c_k(v), out_len >= n*K.
 *   kind PV_EDGE:   out[e*K + (k-k_lo)] = c_k(e), out_len >= m*K, where edge
 *                   id e is the rank of (u,v), u<v, in lexicographic order
 *                   (the order of pv_graph_edge_list).
 * out is host memory.  A range wider than PV_MAX_LOCAL_K (per vertex) or 8
 * (per edge) values of k is counted window by window, one tree walk each;
 * each walk is truncated at its window's largest k hold vertices.  stats
 * describe the last walk.
 * overflow_bits (may be NULL): uint64[1], all bits set if some count is
 * >= 2^128.
 */
pv_status pv_count_local(pv_graph *g, int32_t kind, int32_t k_lo, int32_t k_hi,
                         pv_u128 *out, int64_t out_len, uint64_t *overflow_bits,
                         pv_stats *stats);

/* The edges (u<v) in edge-id order: u[m], v[m] host arrays.  Edge e's
   per-edge counts c_k(e) (Sec. 1.1; Alg. 2 pair steps) are row e of
   pv_count_local's and pv_count's per-edge output. */
pv_status pv_graph_edge_list(pv_graph *g, int32_t *u, int32_t *v);

/*
 * One pass computing global counts (all k, or up to k_max) and, optionally,
 * local counts in the same tree walk.  This is the whole hot path: orient
 * (if `reorient` or not yet oriented), build the SCT, read the counts.
 *   counts/cap/omega_out/overflow_bits: as pv_count_global (host).
 *   local_kind: PV_NONE, PV_VERTEX or PV_EDGE; local_out is DEVICE memory of
 *   (n or m) * (k_hi-k_lo+1) pv_u128, zero-filled by this call.
 *   local_ovf (host, may be NULL): uint64[1] overflow bits of the local range.
 * With k_max <= 0 and local counts requested the tree is not truncated.
 */
pv_status pv_count(pv_graph *g, int32_t reorient, int32_t k_max,
                   pv_u128 *counts, int32_t cap, int32_t *omega_out,
                   uint64_t *overflow_bits,
                   int32_t local_kind, int32_t k_lo, int32_t k_hi,
                   pv_u128 *local_out, uint64_t *local_ovf, pv_stats *stats);

/*
 * Counts restricted to some root children of the SCT.  The root's children
 * N+(v) are independent subproblems (Sec. 5, parallel version: each one is
 * counted with its own counters and the results are summed), and the subtree
 * of N+(v) holds exactly the cliques whose smallest-key vertex is v (Sec. 4,
 * Thm. scr).  Only the subtrees of the given roots (host int32 ids, distinct)
 * are built, so counts[k] is the number of k-cliques whose smallest-key
 * vertex is one of the roots (counts[0] = 0).  Used for sampled checks on
 * graphs whose full count is too large, and to split a count over calls.
 *   local_kind PV_NONE, PV_VERTEX or PV_EDGE: local counts of those cliques
 *   only, for k_lo <= k <= k_hi, into the DEVICE buffer local_out of
 *   (n or m) * (k_hi-k_lo+1) pv_u128 (zero-filled by this call; layout and
 *   limits as pv_count).  local_ovf (host, may be NULL) as pv_count.
 */
pv_status pv_count_roots(pv_graph *g, const int32_t *roots, int32_t nroots, int32_t k_max,
                         pv_u128 *counts, int32_t cap, int32_t *omega_out,
                         uint64_t *overflow_bits, int32_t local_kind, int32_t k_lo, int32_t k_hi,
                         pv_u128 *local_out, uint64_t *local_ovf, pv_stats *stats);

/*
 * Batched counts: G graphs (loaded on this context's device) counted in one
 * launch sequence as their disjoint union.  Root subproblems are
 * independent (Sec. 5, parallel version) and a union's canonical peel orders
 * each graph as it would alone, so every graph's tree and counts are those
 * of a single call; all graphs' subproblems share the device work queues.
 *   counts [G][cap] (host), omega [G] (host, may be NULL),
 *   overflow_bits [G][(cap+63)/64] (host, may be NULL): as pv_count_global
 *   per graph; PV_EBUFSIZE if some graph's omega needs more than cap.
 *   local_kind PV_NONE or PV_VERTEX; local_out is DEVICE memory of
 *   (sum of n) * (k_hi-k_lo+1) pv_u128, graph b's rows first at the sum of
 *   the earlier graphs' n (zero-filled by this call).  Global counts are for
 *   all k (k_max <= 0) or truncated at k_max.
 * The graphs may be used again afterwards; the union is internal scratch.
 */
pv_status pv_count_batch(pv_ctx *ctx, int32_t G, pv_graph *const *gs, int32_t k_max,
                         pv_u128 *counts, int32_t cap, int32_t *omega, uint64_t *overflow_bits,
                         int32_t local_kind, int32_t k_lo, int32_t k_hi, pv_u128 *local_out,
                         uint64_t *local_ovf, pv_status *status, pv_stats *stats);

/* pv_count_batch with global counts only.  status [G] (host, may be NULL):
 * each graph's own status (PV_OK, PV_EBUFSIZE if cap <= its omega,
 * PV_EOVERFLOW if one of its counts reached 2^128); the return value is
 * PV_EBUFSIZE if any graph's is, else PV_EOVERFLOW if any graph's is. */
pv_status pv_count_global_batch(pv_ctx *ctx, int32_t G, pv_graph *const *gs, int32_t k_max,
                                pv_u128 *counts, int32_t cap, int32_t *omega,
                                uint64_t *overflow_bits, pv_status *status, pv_stats *stats);

/* ------------------------------------------------------------ serving
 * A request loop (continuous batching) over graphs that stay resident on
 * the device.  Worker threads, each with its own context and HIP stream,
 * take all pending requests that fit one pass's HBM budget and count them in
 * one pv_count_batch pass; requests that arrive meanwhile go to the next free
 * worker, so passes overlap on the GPU.  Results are identical to one call
 * per request (the union's trees are the graphs' own).
 */
typedef struct pv_server pv_server;

typedef struct {
    int32_t device;       /* HIP device */
    int32_t workers;      /* worker threads (>= 1), one context and stream each */
    int32_t max_batch;    /* most requests in one pass (>= 1) */
    int64_t cache_bytes;  /* device bytes of idle resident graph CSRs kept between requests (LRU);
                             graphs pinned by running passes come on top */
    int64_t batch_bytes;  /* device bytes one pass may use by the admission estimate (its graphs'
                             union copy and orientation, SCT workspace, per-vertex output);
                             larger requests are refused.  A worker context's hard limit is
                             2 * batch_bytes + 64 MiB; a pass that reaches it is split */
} pv_server_cfg;

#define PV_REQ_GLOBAL 0   /* global counts C_k for all k */
#define PV_REQ_VERTEX 1   /* global counts plus c_k(v) for k_lo <= k <= k_hi (at most 8 values) */

typedef struct {
    uint64_t graph_key;       /* names the graph; a resident graph is reused by key */
    int32_t n;                /* host CSR (as pv_graph_load_csr): read during the request's */
    const int32_t *row_ptr;   /* pass when the key is not resident, so it stays valid until */
    const int32_t *col;       /* the request completes; row_ptr[n] is read at submit */
    int32_t kind;             /* PV_REQ_GLOBAL or PV_REQ_VERTEX */
    int32_t k_lo, k_hi;       /* PV_REQ_VERTEX only */
    pv_u128 *counts;          /* host [cap]: counts[k] = C_k (as pv_count_global) */
    int32_t cap;
    pv_u128 *vertex_out;      /* host [n][k_hi-k_lo+1] (PV_REQ_VERTEX only) */
} pv_request;

typedef struct {
    pv_status status;         /* PV_OK, PV_EBUFSIZE (cap too small), PV_EOVERFLOW, PV_ECANCELLED, ... */
    int32_t omega;
    uint64_t overflow;        /* overflow bits of C_0..C_63 */
    uint64_t local_overflow;  /* nonzero if a per-vertex count reached 2^128 */
    double queue_us;          /* submit -> start of its pass */
    double run_us;            /* duration of its pass */
    double total_us;          /* submit -> outputs written and the request complete */
    int32_t batch_size;       /* requests in its pass */
} pv_result;

/* Start the workers.  PV_EINVAL on a bad configuration. */
pv_status pv_server_start(const pv_server_cfg *cfg, pv_server **out);

/* Queue a request (thread-safe).  The outputs are written before the
 * request completes.  PV_ENOMEM if the request alone exceeds batch_bytes. */
pv_status pv_server_submit(pv_server *s, const pv_request *req, uint64_t *ticket);

/* Result of a completed request (its ticket is then retired); PV_EAGAIN if
 * it is not complete (after timeout_us microseconds; < 0 waits forever). */
pv_status pv_server_wait(pv_server *s, uint64_t ticket, int64_t timeout_us, pv_result *out);
pv_status pv_server_poll(pv_server *s, uint64_t ticket, pv_result *out);

/* Cancel a request that is not yet in a pass (its result reports
 * PV_ECANCELLED); PV_EAGAIN if it already runs. */
pv_status pv_server_cancel(pv_server *s, uint64_t ticket);

/* Resident graphs, their device bytes, and requests waiting for a pass. */
pv_status pv_server_stats(pv_server *s, int32_t *resident, int64_t *resident_bytes, int32_t *pending);

/* Finish running passes, cancel queued requests, free everything. */
void pv_server_stop(pv_server *s);

#ifdef __cplusplus
}
#endif

#endif /* PIVOTER_H */
