// Internal declarations shared by the host runtime (api.cpp) and the kernel
// translation units.  Not part of the public ABI (include/pivoter.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pivoter.h"  // PV_MAX_ALPHA and the status codes

struct DevInfo {
    int device;
    int num_cu;
    int lds_per_block;   // bytes of LDS a workgroup may use
    int lds_per_cu;
};

// control block of the peel (zero-filled before a launch,
// minv set to INT_MAX)
struct PeelCtl {
    int cnt[3];          // frontier sizes, rotating by sub-round
    int minv[2];         // smallest remaining degree at a level change
    int subrounds;       // out: number of sub-rounds
    int alpha;           // out: degeneracy (largest level)
    int err;             // out: a grid barrier timed out
    int nlong;           // rows of the solo subgraph split over the grid
    int blk_r, blk_nf, blk_removed;  // where block 0's run of small sub-rounds stopped
    // out, for diagnostics: sub-rounds of the grid phase run by the whole
    // grid, by block 0 alone, level changes of the grid phase, vertices left
    // to the solo phase; the 100 MHz real-time clock at the start, at the
    // end of the grid phase, after the compaction and at the end
    int n_grid, n_block, n_levels, n_solo;
    unsigned long long t_mark[4];
    unsigned bar_flag[256 * 32];  // grid barrier: barriers passed by each block, one 128-byte line each
};

#define PV_PEEL_THREADS 1024
#define PV_PEEL_MAX_BLOCKS 256
// the peel's last PV_SOLO_MAX vertices are finished by one workgroup
// (local ids and remaining degrees below 2^16)
#define PV_SOLO_MAX 16384

struct PeelArgs {
    int n;
    const int *rp, *col;
    int *deg, *sub;      // [n]
    int *fa, *fb;        // frontiers [n]
    PeelCtl *ctl;
    int *lid;            // [n] local id in the solo phase, -1 outside it
    int *uverts;         // [PV_SOLO_MAX] vertex of each local id
    int *ldeg;           // [PV_SOLO_MAX] degree inside the solo subgraph
    int *lrp;            // [PV_SOLO_MAX + 1] local CSR rows
    int *lcol;           // [nnz] local CSR columns
    int *bcnt;           // [blocks] per-block counts
    int *lrow;           // [2 * PV_SOLO_MAX] long rows of U (local ids), then one fill cursor each
};

// Largest out-degree handled by the compact (register) tier.  Roots with
// |N+(v)| <= LIGHT_MAX are built entirely in registers; larger roots start in
// the multi-word tier and drop into the compact tier once |S| <= LIGHT_MAX.
// 62 rather than 64 keeps lanes 62 and 63 free for the per-vertex totals.
#define PV_LIGHT_MAX 62

// Largest node set walked by the lane tier (one subtree per lane, up to 64
// at once per wave); its rows are 8-bit masks.
#define PV_LANE_MAX 8

// ------------------------------------------------------------- item types

// Compact-tier subproblem (32 bytes), one of two kinds:
//   node item  (uni bit 31 clear): the SCT node S with hold / pivot members
//              H, P inside the universe; hp = h | p << 16 (path totals)
//   frame item (uni bit 31 set): an unfinished node whose pivot child is
//              done; S is its set with the visited hold children removed,
//              hp = pivot | h << 6 | p << 19 as on the walk's stack
struct CItem {
    uint64_t S, H, P;
    uint32_t uni;
    uint32_t hp;
};

// Persistent walk: one launch takes every unit (roots, multi-word items,
// compact node and frame items) from device queues until the whole tree is
// walked.  The compact queue is split into PV_QSLICES slices, each with its
// own claim and reservation counters on their own 128-byte lines (a wave
// pushes to its home slice and claims from it first, then from the
// others); the multi-word queue has one.  Queue storage is linear: slice s
// of the compact queue is c_out[s * c_scap, (s + 1) * c_scap).
#define PV_QSLICES 8
struct alignas(128) PvLine {
    unsigned long long v;
};
struct PersistCtl {
    PvLine done;              // units finished (roots, items, unused slots), added by waves going idle
    PvLine state;             // error bits: 1 no progress for 10 s, 2 a published slot never came
    PvLine abort;             // set by the host: waves stop taking units
    PvLine chead[PV_QSLICES];  // next slot to claim, per slice (int in .v)
    PvLine ctail[PV_QSLICES];  // slots reserved by producers, per slice (may pass capacity)
    PvLine mhead, mtail;       // the multi-word queue
};

struct LevelArgs {
    // graph
    int n;
    const int *orow, *ocol, *order;
    int heavy_base, nheavy;  // level 0: heavy roots order[heavy_base, +nheavy)
    int light_base, nlight;  // level 0: light roots order[light_base, +nlight)
    int kmax, dfs_max;
    int dfs_budget;          // nodes a wave walks depth first before splitting
    int lane_max;            // nodes with |S| <= lane_max go to the lane tier (0: off)
    // level input
    int level;
    int n_mw_in, n_c_in;
    const uint64_t *mw_in;   // stride mw_stride u64
    const CItem *c_in;
    // level output
    uint64_t *mw_out;
    CItem *c_out;
    int *mw_out_n, *c_out_n;
    int mw_cap, c_cap;
    int mw_stride;           // 3W + 1
    // heavy universes (indexed by heavy root rank)
    uint64_t *hu_rows;       // [nheavy][W][dpad]
    int *hu_vl;              // [nheavy][dpad]
    int W, dpad;
    // compact universes
    uint64_t *u_rows;        // [cap][64]
    int *u_gid;              // [cap][64]   (local counts only)
    int2 *u_pref;            // [cap] {offset, length} into pref pool (local only)
    int *u_n, u_cap;
    // prefix entries: the root's id, then hold / pivot vertices (bit 31 set
    // for a pivot); per vertex, those of a multi-word universe are local
    // indices into N+(root), per edge they are vertex ids
    int *pref_pool, *pref_n, pref_cap;
    int *u_grp;              // [cap] per vertex: the heavy-root index of a multi-word universe, else -1
    // work cursors, one per unit kind.  A claim takes chunk c < nch[kind]:
    // units c, c + nch, c + 2 nch, ... below n0[kind]; claims past nch take
    // one unit each from n0 on
    int *next;
    int n0[3], nch[3];
    // outputs
    unsigned long long *hist;
    int hd;
    unsigned long long *counters;  // PV_NCOUNTERS slots: nodes, leaves, work, -, work per unit kind [3],
                                   // child work, leaf sum of h + p, leaf sum of p + 1
    int *flags;                    // bit0: buffer overflow, bit2: edge id lookup failed,
                                   // bit3: an invariant of the walk failed (checked builds)
    int *check;                    // checked builds: source line of the first failed invariant
    // local counts
    uint64_t *vout;                // [n][kstride] (per vertex) or [m][kstride] (per edge) u128;
                                   // this pass writes columns 0..K-1
    int klo, K, kstride;
    const uint64_t *bin_pad;       // padded 64-bit binomials, rows tab_stride apart, see VertexSink
    const uint64_t *bin_pad_hi;    // their high limbs (nullptr when every binomial used fits 64 bits)
    const uint8_t *bin_bad;        // [bin_bn][bin_bn]: C(a, b) >= 2^128
    int bin_bn;
    int tab_stride;
    int *lovf;
    // per-edge counts: edge ids and the universes' prefix-pair sums
    const int *sub;                // peel sub-round of every vertex (the orientation key)
    const int *o2e;                // [m] oriented CSR position -> edge id
    uint64_t *umem;                // [u_cap][64][2][K] u128: member sums toward H / P prefix
    uint64_t *utot;                // per edge [u_cap][3][K] u128: HH, HP, PP sums; per vertex
                                   // [u_cap][2][K]: totals owed to hold / pivot prefix vertices
    int *ueid;                     // [u_cap][64][64] edge id of each member pair of a universe
    int *weid;                     // [waves of a light-root launch][64][64] the same per wave
    uint64_t *escr;                // [waves][2][64][2][K] u128: join snapshots and finished-stay
                                   // sums of the path members; the kinds of a level run
                                   // concurrently, so kind m's waves start at escr_wave0[m]
    int escr_wave0[3];
    // local counts known to stay below 2^62: the additions (a vertex's sums,
    // an edge's pair charges) go to 32-bit halves, two values of k per 64-bit
    // word (nullptr: straight to vout).  epk [rows][kws] words (rows: n or
    // m), the first kw = ceil(K / 2) used, k = 2i in the low half and 2i + 1
    // in the high half (kws, a power of two, keeps a row's words in one
    // 64-byte line); ewrap [rows][kws]: carries out of the low half (low 32
    // bits) and out of the word (high 32 bits), counted
    uint64_t *epk;
    uint64_t *ewrap;
    int kw, kws;
    // batches (a disjoint union of graphs): graph of every vertex, nullptr
    // for a single graph; hist then holds one hd*hd histogram per graph
    const int *vgraph;
    int *u_root;                   // [u_cap] root vertex of each universe (batch only)
    // persistent walk (unit kind PV_UNITS_ALL); persist = 0: level by level
    int persist;
    // phase times per unit kind ([3][16] ticks), filled by builds with
    // PV_PHASE_TIMING only (nullptr: off)
    unsigned long long *phase;
    // the call's abort flag (nonzero: hand out no more units); nullptr: none
    const int *abort;
    PersistCtl *pctl;
    int *cready, *mready;          // per queue slot: 0 not yet written, 1 written, 2 never written
    int c_scap, m_cap;             // compact slots per slice; multi-word slots
};


hipError_t pv_launch_check_rowptr(int n, long long nnz, const int *rp, int *d_err, hipStream_t s);
hipError_t pv_launch_validate(int n, long long nnz, const int *rp, const int *col, int *d_err, hipStream_t s);
hipError_t pv_launch_peel(const DevInfo &dev, const PeelArgs &pa, hipStream_t s);
// row_tmp: nnz ints of scratch (N+(v) staged at rp[v])
// rows longer than this are walked by a whole workgroup when the orientation
// counts out-degrees (a hub's row would hold one wave for its whole length)
#define PV_ORIENT_BLOCK_ROW 4096
hipError_t pv_launch_orient(const DevInfo &dev, int n, const int *rp, const int *col, const int *sub,
                            int *odeg, int *orow, int *ocol, int *alpha, int *scan_tmp, int *row_tmp,
                            int *wide, hipStream_t s);  // wide: [1 + nnz / PV_ORIENT_BLOCK_ROW] ints
// roots by out-degree, largest first; bh: chunks * (PV_MAX_ALPHA + 1) ints
hipError_t pv_launch_root_order(int n, const int *amax, const int *odeg, int *bh, int chunks,
                                int *order, int *bounds, int light_max, hipStream_t s);
// out-degree histogram in powers of two: bucket 0 holds d = 0, bucket b > 0
// holds 2^(b-1) <= d < 2^b (last bucket: everything above); hist zeroed by
// the caller
#define PV_DEG_BUCKETS 16
hipError_t pv_launch_deg_hist(int n, const int *odeg, int *hist, hipStream_t s);
// chunks of the root ordering for n vertices
static inline int pv_root_chunks(int n) {
    const int c = (n + 4095) / 4096;
    return c < 1 ? 1 : (c > 1024 ? 1024 : c);
}

// SCT build + leaf read-off
// unit kinds of a level launch
#define PV_UNITS_MW 0
#define PV_UNITS_ITEMS 1
#define PV_UNITS_LIGHT 2
#define PV_UNITS_ALL 3   // the persistent walk: every kind from the device queues

// slots of the level kernel's work counters
#define PV_NCOUNTERS 12
#define PV_CTR_CHILD 8
#define PV_CTR_HP 9
#define PV_CTR_PP 10
// `a` is a device pointer to the launch arguments
// local-count kinds of the level kernel: per vertex with u128 or u64 per-visit
// accumulators, or per edge
#define PV_LK_VERTEX128 0
#define PV_LK_EDGE 1
#define PV_LK_VERTEX64 2
hipError_t pv_launch_level(const LevelArgs *a, int kl, int lk, int mode, int blocks, hipStream_t s);
int pv_level_blocks_per_cu(int kl, int lk, int mode);
hipError_t pv_launch_edge_prefix(const LevelArgs *a, int blocks, hipStream_t s);
// adds the packed local table (rows of kw words, kws apart) to vout's K columns
hipError_t pv_launch_local_unpack(const uint64_t *epk, const uint64_t *ewrap, long long m, int kw, int kws, int K,
                                 uint64_t *vout, int kstride, uint32_t bias, int num_cu, hipStream_t s);
// per-vertex prefix sums, grouped by heavy root (max_units >= universes made;
// ngroups = number of heavy roots; rows: N+(root) rows summed per LDS pass,
// at most PV_PREFIX_SLOTS / K - 1)
#define PV_PREFIX_SLOTS 2048
#define PV_PREFIX_SLICE 64
struct PrefixWork {
    int *gcnt, *goff, *gpos, *glist, *scan_tmp;  // [ngroups], [ngroups+1], [u_cap], [u_cap], scan temp
};
hipError_t pv_launch_vertex_prefix(const LevelArgs *a, int max_units, int ngroups, const PrefixWork &w,
                                   int rows, hipStream_t s);
// counts in W 64-bit limbs.  phase 0: *span = largest h + p of a nonzero
// bin (span zeroed by the caller).  phase 1: table tab [bn][bn][tl] of C(p, j)
// (tl limbs, bn = span + 1) and out [kcap][W] (W = tl + 1), omega as the
// largest k with a nonzero count (zeroed by the caller)
hipError_t pv_launch_count_wide(const unsigned long long *hist, int hd, int kcap, int kmax, int c0, int *span,
                                uint64_t *tab, int bn, int tl, int W, uint64_t *out, int *omega, int phase,
                                hipStream_t s);
// frequency distribution of one column of a [rows][K] u128 table: keys
// [npad][2] (npad = power of two >= rows), flags / idx / pos [rows + 1],
// vals [rows][2], scan_tmp rows / 1024 + 2 ints; after the launch idx[rows]
// is the number of distinct values D, vals[0..D) the values in increasing
// order and pos[0..D) the sorted position of each value's first row
struct FreqWork {
    uint64_t *keys, *vals;
    int *flags, *idx, *pos, *scan_tmp;
};
hipError_t pv_launch_frequency(const uint64_t *src, int rows, int K, int col, long long npad, const FreqWork &w,
                               hipStream_t s);
// exclusive scan: out[i] = sum_{j<i} in[j] for i <= n; tmp: n / 1024 + 2 ints
hipError_t pv_launch_excl_scan(int n, const int *in, int *tmp, int *out, hipStream_t s);
// per-edge ids: o2e[q] = lexicographic id of the edge at oriented position q
hipError_t pv_launch_edge_ids(const DevInfo &dev, int n, const int *rp, const int *col, const int *sub,
                              const int *orow, int *ucnt, int *up, int *o2e, int *scan_tmp,
                              hipStream_t s);
hipError_t pv_launch_sink_roots(int n, const int *order, const int *bounds, unsigned long long *hist,
                                int hd, unsigned long long *counters, uint64_t *vout, int klo, int kstride,
                                const int *vgraph, hipStream_t s);
hipError_t pv_launch_binomials(int bn, uint64_t *tab128, uint8_t *bad, uint64_t *tab64, int *fits64,
                               hipStream_t s);
// pad: 2 (bn + 1) ts words, low limbs then high limbs (all ones where C >= 2^128)
hipError_t pv_launch_binom_pad(int bn, int ts, const uint64_t *tab128, const uint8_t *bad, uint64_t *pad,
                               hipStream_t s);
hipError_t pv_launch_finalize(const unsigned long long *hist, int hd, const uint64_t *tab128,
                              const uint8_t *bad, int bn, int kcap, int kmax, int c0,
                              uint64_t *counts, uint64_t *ovf_words, int *omega, int graphs,
                              hipStream_t s);
// the same on the device's static scratch array (no allocation): after the
// launches *vals holds the D distinct values, *freq their multiplicities and
// (*idx)[rows] = D.  pv_freq_static_init resolves the array's address, once
// per device, with that device current; rows, npad <= PV_FREQ_STATIC_ROWS.
hipError_t pv_freq_static_init(int device);
hipError_t pv_launch_frequency_static(int device, const uint64_t *src, int rows, int K, int col, long long npad,
                                      uint64_t **vals, uint64_t **freq, int **idx, hipStream_t s);
// counters[PV_CTR_HP] += sum over leaves of h + p, counters[PV_CTR_PP] +=
// sum over leaves of p + 1, from graphs [hd][hd] leaf histograms
hipError_t pv_launch_leaf_moments(const unsigned long long *hist, int hd, int graphs,
                                  unsigned long long *counters, hipStream_t s);
// peak microbenchmarks (PV_PEAK_BLOCKS workgroups of 256; sinks hold one
// word per thread)
#define PV_PEAK_BLOCKS 2048
#define PV_PEAK_LDS_READS 15  // 64-bit LDS reads per thread and iteration
hipError_t pv_launch_peak_copy(const void *src, void *dst, long long bytes, hipStream_t s);
hipError_t pv_launch_peak_read(const void *src, long long bytes, unsigned *sink, hipStream_t s);
hipError_t pv_launch_peak_lds(int iters, int zero, unsigned long long *sink, hipStream_t s);
hipError_t pv_launch_peak_valu(int iters, unsigned seed, unsigned *sink, hipStream_t s);
// batches: concatenate graphs into one disjoint union (device descriptors)
struct BatchPart {
    const int *rp, *col;   // the part's own CSR (device)
    int n, voff;           // its vertices and their offset in the union
    long long eoff, nnz;   // its column entries and their offset in the union
};
hipError_t pv_launch_concat(const BatchPart *parts, int G, int maxn, int *rp, int *col, int *vgraph,
                            hipStream_t s);
