// Succinct Clique Tree build and leaf read-off on CDNA (gfx950).
//
// What is computed (Sec. 4, Alg. 1; Sec. 5, Alg. 2 and the depth-first form
// in the proof of Thm. main): every root child N+(v) of the SCT is expanded
// by pivoting -- a node S picks the pivot p in S with the most neighbours in
// S (ties: smallest id), has the pivot child N(S,p) and, for the
// non-neighbours v_1 < v_2 < ... of p in S (p excluded), the hold children
// N(S,v_i) minus {v_1..v_{i-1}}.  A leaf whose path holds h hold and p pivot
// vertices adds C(p, k-h) to C_k (and the per-vertex terms of Alg. 2).
//
// How it is laid out on the GPU:
//   * A subproblem lives in a *universe*: the ordered vertex list of some
//     root's out-neighbourhood (or a subset of it) with the induced
//     adjacency as bit rows.  Sets are bitsets over the universe, and the
//     universe order is vertex-id order, so "smallest id" is "lowest bit".
//   * Compact tier (|universe| <= 64): lane j of a wave holds row j in a
//     64-bit register.  Pivot = wave max of popcount(row & S) (DPP), child
//     sets come from v_readlane of one row, and the DFS stack lives in
//     lane-indexed registers (frame t in lane t).  No LDS on the hot path.
//   * Multi-word tier (|S| > 64, heavy roots only): lane w holds word w of
//     each set; the universe's rows live in HBM, word-major.
//   * Work is split level by level, in the spirit of Alg. 1's breadth-first
//     queue: an item follows its pivot chain (pivot children stay in the
//     same wave) and emits its hold children as items of the next level.
//     Once |S| <= dfs_max the remaining subtree is walked depth first in
//     registers; its size is bounded by the worst case O(3^{s/3}) of
//     Thm. main-BK, so no wave is left with a huge subtree.
//   * Leaves are counted by (h, p) in per-lane registers and folded into a
//     u64 histogram; C_k = sum L[h][p] C(p, k-h) is formed exactly in u128
//     by the finalize kernel.  Per-vertex counts accumulate per member lane
//     in u128 registers and are flushed with carry-exact 64-bit atomics.
#include "common.h"
#include "internal.h"

#define WAVES_PER_BLOCK 4

// Checked builds (-DPV_CHECKED): invariants of the walk are tested on the
// device -- a node's pivot lies in its set, the set, hold and pivot members
// are disjoint, a universe's adjacency is symmetric without loops, stacks
// stay within their frames, and a leaf's (h, p) bin lies in the histogram.
// A failure sets bit 3 of the walk's flag word and keeps the source line of
// the first one; the kernel runs on to its normal end and the host reports
// the line.  Other builds compile the checks out (the condition is not
// evaluated).
#ifdef PV_CHECKED
__device__ __noinline__ void pv_check_failed(int *flags, int *line_out, int line) {
    atomicOr(flags, 8);
    atomicCAS(line_out, 0, line);
}
#define PV_ASSERT(flags, line_out, cond)                                      \
    do {                                                                      \
        if (!(cond)) pv_check_failed((flags), (line_out), __LINE__);          \
    } while (0)
#else
#define PV_ASSERT(flags, line_out, cond) \
    do {                                 \
    } while (0)
#endif

// ------------------------------------------------------------------ sinks

// Global counts: leaf (h,p) -> L[h][p] += 1.  The workgroup keeps the bins
// h < lds_h, p < 64 as u64 counters in LDS (one LDS atomic per leaf, no
// hot global addresses: in dense cores most leaves share a handful of (h,p)
// bins); rarer leaves go straight to the device histogram.  The LDS bins
// are added to the device histogram when the workgroup ends.  lds_h is 32,
// or 16 in the kernels whose lane-tier member slots need the LDS (so that
// four workgroups fit a CU).
#define PV_LDS_H 32
//
// A batch of graphs is counted as one disjoint union: every graph has its
// own histogram (stride hd*hd), and a wave sets the graph of each unit it
// takes.  The workgroup's LDS bins are not used then (a workgroup's units
// come from many graphs); leaves go straight to the graph's histogram.
typedef __attribute__((address_space(3))) unsigned long long lds_u64;

struct GlobalSink {
    lds_u64 *bins;              // LDS [lds_h][64], shared by the workgroup
    unsigned long long *hist;   // wave-uniform copies of the arguments
    unsigned long long *ghist;  // batch: the current graph's histogram
    const int *vgraph;          // batch: graph of every vertex (nullptr: one graph)
    int hd, lds_h;
    unsigned long long leaves;
#ifdef PV_CHECKED
    int *chk_flags, *chk_line;
#endif

    __device__ void init(const LevelArgs &a, unsigned long long *lds_bins, int rows) {
#ifdef PV_CHECKED
        chk_flags = a.flags;
        chk_line = a.check;
#endif
        // an LDS-typed pointer: the bin update is a ds_add, not a flat atomic
        bins = (lds_u64 *)lds_bins;
        lds_h = rows;
        hist = (unsigned long long *)uniform64((uint64_t)a.hist);
        vgraph = (const int *)uniform64((uint64_t)a.vgraph);
        hd = uniformi(a.hd);
        ghist = hist;
        leaves = 0;
    }

    // batch: the unit being walked belongs to the graph of vertex v
    __device__ __forceinline__ void set_vertex(int v) {
        if (vgraph) ghist = hist + (long long)uniformi(vgraph[v]) * hd * hd;
    }

    __device__ void add_leaves(uint32_t k, int) { leaves += k; }

    __device__ __forceinline__ void leaf(int h, int p, int lane) {
        PV_ASSERT(chk_flags, chk_line, h >= 0 && p >= 0 && h + p < hd);
        if (vgraph) {
            if (lane == 0) atomicAdd(&ghist[(long long)h * hd + p], 1ull);
        } else if (h < lds_h && p < 64) {
            if (lane == 0)
                __hip_atomic_fetch_add(&bins[h * 64 + p], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else if (lane == 0) {
            atomicAdd(&hist[(long long)h * hd + p], 1ull);
        }
    }

    // a leaf of one lane's own subtree (lane tier): every lane its own (h,p)
    __device__ __forceinline__ void leaf_lane(int h, int p) {
        PV_ASSERT(chk_flags, chk_line, h >= 0 && p >= 0 && h + p < hd);
        if (vgraph)
            atomicAdd(&ghist[(long long)h * hd + p], 1ull);
        else if (h < lds_h && p < 64)
            __hip_atomic_fetch_add(&bins[h * 64 + p], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else
            atomicAdd(&hist[(long long)h * hd + p], 1ull);
    }
};

// Load through the constant address space: uniform addresses become scalar
// (s_load) loads instead of vector loads with full memory latency.  Only for
// data no wave writes during the launch (the scalar cache does not see
// vector stores): the binomial table.
__device__ __forceinline__ uint64_t ldc64(const uint64_t *p) {
    return *(const __attribute__((address_space(4))) uint64_t *)(uintptr_t)p;
}

// Eight consecutive table entries in one scalar load (s_load_dwordx16; the
// scalar unit needs only dword alignment).  Callers keep p + 8 inside the
// table: every row segment read here is followed by at least one more row.
typedef uint64_t u64x8 __attribute__((ext_vector_type(8)));
typedef u64x8 u64x8_a8 __attribute__((aligned(8)));
__device__ __forceinline__ u64x8 ldc64x8(const uint64_t *p) {
    return *(const __attribute__((address_space(4))) u64x8_a8 *)(uintptr_t)p;
}

// Per-vertex counts (Alg. 2 steps ht and pt).  Lane j < 62 accumulates the
// contributions of universe member j for k = klo..klo+K-1 (members sit on
// lanes 0..61: compact universes hold at most PV_LIGHT_MAX = 62 vertices).
// Lane 62 accumulates what every hold vertex above the universe is owed
// (sum of C(p, k-h)) and lane 63 what every pivot vertex above it is owed
// (sum of C(p-1, k-h-1)), with the same instructions as a member.
//
// Binomials come from a padded table: row a (a = -1..alpha) holds C(a, j)
// for j = -16..ts-17 at [(a + 1) * ts + j + 16] (ts = a.tab_stride, at
// least k_hi + 24), zero outside 0 <= j <= a, so the K values of a leaf are
// one contiguous, range-check-free segment.  Output rows are kstride slots
// apart (a window of a wider k range writes its own columns).
//
// WIDE = false keeps one 64-bit word per slot: the host picks it when a
// wave's sums for one universe visit cannot reach 2^64 (a visit reaches at
// most dfs_budget plus two pivot chains of leaves, each adding a binomial
// of at most C(alpha, k_hi - 1)); the flush widens to u128.
template <int KL, bool WIDE>
struct VertexSink {
    uint64_t lo[KL > 0 ? KL : 1], hi[(KL > 0 && WIDE) ? KL : 1];
    // wave-uniform copies of the arguments
    const uint64_t *tab;
    const uint64_t *tabh;    // high limbs of the table (nullptr: every binomial used fits 64 bits)
    const uint8_t *bad;      // [bn][bn]: C(a, b) >= 2^128
    bool wrapped;            // a 128-bit sum of this lane wrapped (with the wide table only)
    uint64_t *vout;
    uint64_t *epk, *ewrap;   // packed 32-bit halves (64-bit sums only; nullptr: additions go to vout)
    uint64_t *utot;  // [u_cap][2][K]: what the hold / pivot vertices above a universe are owed
    const int *pool;
    int *lovf;
    int klo, K, khi, ks, ts, bn, kw, kws;

    __device__ void init(const LevelArgs &a, uint64_t *, int) {
        tab = (const uint64_t *)uniform64((uint64_t)a.bin_pad);
        tabh = WIDE ? (const uint64_t *)uniform64((uint64_t)a.bin_pad_hi) : nullptr;
        bad = (const uint8_t *)uniform64((uint64_t)a.bin_bad);
        bn = uniformi(a.bin_bn);
        vout = (uint64_t *)uniform64((uint64_t)a.vout);
        epk = WIDE ? nullptr : (uint64_t *)uniform64((uint64_t)a.epk);
        ewrap = (uint64_t *)uniform64((uint64_t)a.ewrap);
        kw = uniformi(a.kw);
        kws = uniformi(a.kws);
        utot = (uint64_t *)uniform64((uint64_t)a.utot);
        pool = (const int *)uniform64((uint64_t)a.pref_pool);
        lovf = (int *)uniform64((uint64_t)a.lovf);
        klo = uniformi(a.klo);
        K = uniformi(a.K);
        khi = klo + K - 1;
        ks = uniformi(a.kstride);
        ts = uniformi(a.tab_stride);
        reset();
    }

    __device__ void reset() {
#pragma unroll
        for (int i = 0; i < KL; i++) {
            lo[i] = 0;
            if (WIDE) hi[i] = 0;
        }
        wrapped = false;
    }

    __device__ __forceinline__ uint64_t hiw(int i) const { return WIDE ? hi[i] : 0ull; }

    // path bookkeeping is only needed for pairs (EdgeSink)
    __device__ __forceinline__ void set_table(const int *) {}
    __device__ __forceinline__ const int *etab_ptr() const { return nullptr; }
    __device__ __forceinline__ void begin(uint64_t, uint64_t, int) {}
    __device__ __forceinline__ void join(int, uint64_t, uint64_t, bool, int) {}
    __device__ __forceinline__ void join_set(uint64_t, uint64_t, uint64_t, int) {}
    __device__ __forceinline__ void leave(uint64_t, uint64_t, uint64_t, int, int) {}

    __device__ __forceinline__ void leaf(int h, int p, uint64_t H, uint64_t P, int lane,
                                         const LevelArgs &) {
        // nothing for k <= khi when h > khi (every clique of the leaf has
        // at least h vertices), nor when h + p < klo
        if (h > khi || h + p < klo) return;
        const bool inH = ((H >> lane) & 1) || lane == 62;
        const bool inP = ((P >> lane) & 1) || lane == 63;
        const uint64_t *rowH = tab + (p + 1) * ts + (klo - h + 16);  // C(p, k-h)
        const uint64_t *rowP = tab + p * ts + (klo - h + 15);        // C(p-1, k-h-1)
        constexpr int NC = KL > 0 ? (KL + 7) / 8 : 1;
        u64x8 vH[NC], vP[NC];
#pragma unroll
        for (int c = 0; c < (KL + 7) / 8; c++) {
            vH[c] = ldc64x8(rowH + 8 * c);
            vP[c] = ldc64x8(rowP + 8 * c);
        }
        // every slot accumulates (slots >= K read in-table entries and are
        // never flushed), so no per-slot guard; a lane takes the hold or the
        // pivot binomial through masks
        uint64_t mH = inH ? ~0ull : 0ull;
        uint64_t mP = (!inH && inP) ? ~0ull : 0ull;
        // keep the masks as opaque vector values: the AND/OR form then takes
        // the scalar binomials as direct operands (no per-slot moves/selects)
        asm volatile("" : "+v"(mH), "+v"(mP));
        if (WIDE && tabh) {
            // binomials beyond 64 bits: the high limbs from the second table
            const long long hoff = tabh - tab;
            u64x8 uH[NC], uP[NC];
#pragma unroll
            for (int c = 0; c < (KL + 7) / 8; c++) {
                uH[c] = ldc64x8(rowH + hoff + 8 * c);
                uP[c] = ldc64x8(rowP + hoff + 8 * c);
            }
#pragma unroll
            for (int kk = 0; kk < KL; kk++) {
                const uint64_t v = (vH[kk / 8][kk % 8] & mH) | (vP[kk / 8][kk % 8] & mP);
                const uint64_t u = (uH[kk / 8][kk % 8] & mH) | (uP[kk / 8][kk % 8] & mP);
                lo[kk] += v;
                const uint64_t h0 = hi[kk], c = (lo[kk] < v) ? 1ull : 0ull;
                hi[kk] = h0 + u + c;
                if (kk < K) wrapped |= hi[kk] < h0 || (hi[kk] == h0 && (u | c) != 0);
            }
            // every C(a, b) with a <= 131 fits 128 bits; from p = 132 on a
            // leaf may need one that does not (its counts then overflow)
            if (p >= 132) overflow_check(h, p);
            return;
        }
#pragma unroll
        for (int kk = 0; kk < KL; kk++) {
            const uint64_t v = (vH[kk / 8][kk % 8] & mH) | (vP[kk / 8][kk % 8] & mP);
            lo[kk] += v;
            if (WIDE) hi[kk] += (lo[kk] < v) ? 1ull : 0ull;
        }
    }

    // a leaf with p >= 132 pivots: does some k of the range need a binomial
    // that reaches 2^128?  (C(p, k-h) for hold vertices, C(p-1, k-h-1) for
    // pivot vertices; wave-uniform, rare)
    __device__ void overflow_check(int h, int p) {
        bool big = false;
        for (int k = klo; k <= khi; k++) {
            const int j = k - h;
            if (j >= 0 && j <= p && p < bn) big |= bad[(long long)p * bn + j] != 0;
            if (j >= 1 && j - 1 <= p - 1 && p - 1 < bn) big |= bad[(long long)(p - 1) * bn + j - 1] != 0;
        }
        if (big && lane_id() == 0) atomicOr(lovf, 1);
    }

    // lane tier: add x to slot kk
    __device__ __forceinline__ void add_val(int kk, uint64_t x) {
#pragma unroll
        for (int i = 0; i < KL; i++) {
            if (i == kk) {
                lo[i] += x;
                if (WIDE) hi[i] += (lo[i] < x) ? 1ull : 0ull;
            }
        }
    }

    // lane tier: move the sums into this member's LDS slots (zero between
    // batches) so that no register holds them while the lanes walk; the
    // batch's own additions land on top and add_slots takes them all back
    __device__ __forceinline__ void park(lds_u64 *slot) {
        if constexpr (!WIDE) {
#pragma unroll
            for (int kk = 0; kk < KL; kk++) {
                slot[kk] = lo[kk];
                lo[kk] = 0ull;
            }
        }
    }

    // lane tier: add this member's LDS slots and clear them
    __device__ __forceinline__ void add_slots(lds_u64 *slot, int) {
#pragma unroll
        for (int kk = 0; kk < KL; kk++) {
            const uint64_t v = slot[kk];
            slot[kk] = 0ull;
            lo[kk] += v;
            if (WIDE) hi[kk] += (lo[kk] < v) ? 1ull : 0ull;
        }
    }

    // Member vertex gid's sums in the packed table: the values of k = 2i and
    // 2i + 1 added to word i's 32-bit halves with one 64-bit atomic (all
    // words first, so that their latencies overlap), then the carries out of
    // each half, read off the old words, counted in ewrap (the table is
    // added to vout after the walk).  A sum of 2^32 or more goes to vout.
    __device__ __forceinline__ void flush_packed(int gid) {
        constexpr int KWL = KL > 0 ? (KL + 1) / 2 : 1;
        uint64_t old[KWL], x[KWL];
#pragma unroll
        for (int i = 0; i < KWL; i++) {
            old[i] = 0ull;
            x[i] = 0ull;
            if (i < kw) {
                const uint64_t v0 = lo[2 * i], v1 = (2 * i + 1 < K) ? lo[(2 * i + 1) % KL] : 0ull;
                if (((v0 | v1) >> 32) == 0) {
                    x[i] = v0 | (v1 << 32);
                    if (x[i]) old[i] = atomicAdd((unsigned long long *)(epk + (long long)gid * kws + i),
                                                 (unsigned long long)x[i]);
                } else {
                    uint64_t *dst = vout + 2 * ((long long)gid * ks + 2 * i);
                    if (v0) (void)atomic_add_u128(dst, v0, 0ull);
                    if (v1) (void)atomic_add_u128(dst + 2, v1, 0ull);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < KWL; i++) asm volatile("" : "+v"(old[i]));
#pragma unroll
        for (int i = 0; i < KWL; i++) {
            if (x[i]) {
                const uint64_t c0 = ((old[i] & 0xffffffffull) + (x[i] & 0xffffffffull)) >> 32;
                const uint64_t c1 = (old[i] + x[i] < old[i]) ? 1ull : 0ull;
                if (c0 | c1)
                    atomicAdd((unsigned long long *)(ewrap + (long long)gid * kws + i),
                              (unsigned long long)(c0 | (c1 << 32)));
            }
        }
    }

    // members: lane j < nm owns vertex gid; above the universe: `root` (a
    // light root walked without a universe in memory, a hold vertex) or, with
    // a universe, the totals go to its accumulators (a final kernel adds them
    // to every vertex of its prefix once)
    __device__ void flush(int lane, int nm, int gid, int root, int2, int uni, const LevelArgs &) {
        bool ovf = WIDE && ballot64(wrapped && (lane < nm || lane >= 62)) != 0;
        if (!WIDE && epk) {
            if (lane < nm) flush_packed(gid);
        } else if (lane < nm) {
            // the low-limb adds of all slots first, so that their latencies
            // overlap; then the (rare) carries and the high limbs
            uint64_t old[KL > 0 ? KL : 1];
#pragma unroll
            for (int kk = 0; kk < KL; kk++)
                old[kk] = (kk < K) ? atomic_add_u128_lo(vout + 2 * ((long long)gid * ks + kk), lo[kk]) : 0ull;
            // the returned limbs are first needed here (keeps the compiler
            // from waiting for each atomic inside its own branch)
#pragma unroll
            for (int kk = 0; kk < KL; kk++) asm volatile("" : "+v"(old[kk]));
#pragma unroll
            for (int kk = 0; kk < KL; kk++)
                if (kk < K) ovf |= atomic_add_u128_hi(vout + 2 * ((long long)gid * ks + kk), lo[kk], old[kk], hiw(kk));
        }
        root = uniformi(root);
        uni = uniformi(uni);
        if (root >= 0 || uni >= 0) {
            // lane kk < K takes the owed totals for k = klo + kk from lanes 62/63
            uint64_t thl = 0, thh = 0, tpl = 0, tph = 0;
#pragma unroll
            for (int kk = 0; kk < KL; kk++) {
                if (kk < K) {
                    const uint64_t a = readlane64(lo[kk], 62), b = WIDE ? readlane64(hiw(kk), 62) : 0ull;
                    const uint64_t c = readlane64(lo[kk], 63), d = WIDE ? readlane64(hiw(kk), 63) : 0ull;
                    if (lane == kk) {
                        thl = a;
                        thh = b;
                        tpl = c;
                        tph = d;
                    }
                }
            }
            if (lane < K) {
                if (root >= 0) {
                    if (thl | thh) ovf |= atomic_add_u128(vout + 2 * ((long long)root * ks + lane), thl, thh);
                } else {
                    uint64_t *ut = utot + 2 * ((long long)uni * 2 * K + lane);
                    uint64_t oh = atomic_add_u128_lo(ut, thl), op = atomic_add_u128_lo(ut + 2 * K, tpl);
                    asm volatile("" : "+v"(oh), "+v"(op));
                    ovf |= atomic_add_u128_hi(ut, thl, oh, thh);
                    ovf |= atomic_add_u128_hi(ut + 2 * K, tpl, op, tph);
                }
            }
        }
        if (ovf) atomicOr(lovf, 1);
        reset();
    }
};


// Edge id of the edge {x, y} (both endpoints given as vertex ids): the
// edge is stored once in the oriented CSR, at its smaller-key end, and o2e
// maps that position to the lexicographic edge id.  -1 if x, y are not
// adjacent (never the case for pairs of one root-to-leaf path).
__device__ __forceinline__ int edge_id(int x, int y, const int *__restrict__ sub,
                                       const int *__restrict__ orow, const int *__restrict__ ocol,
                                       const int *__restrict__ o2e) {
    const int sx = sub[x], sy = sub[y];
    int u = x, w = y;
    if (sy < sx || (sy == sx && y < x)) {
        u = y;
        w = x;
    }
    int lo = orow[u], hi = orow[u + 1];
    const int end = hi;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ocol[mid] < w) lo = mid + 1;
        else hi = mid;
    }
    return (lo < end && ocol[lo] == w) ? o2e[lo] : -1;
}

// Per-edge counts (Alg. 2 steps for pairs): a leaf with h hold and p pivot
// vertices adds, for k = klo..khi,
//     C(p, k-h)      to every pair of hold vertices          (type HH)
//     C(p-1, k-h-1)  to every hold/pivot pair                (type HP)
//     C(p-2, k-h-2)  to every pair of pivot vertices         (type PP).
// Instead of touching every pair at every leaf, a pair is charged once per
// stay of its later-joined end j on the walk's path: the partners above j
// stay on the path for all of j's stay, and the leaves of a stay are a
// contiguous run of the depth-first order.  The wave keeps running sums T
// of each type over the leaves it has visited (lane kk holds slot k = klo +
// kk), each member records T when it joins (a snapshot in per-wave scratch
// memory), and its stay owes T - snapshot: toward hold partners the type
// (H, role of j), toward pivot partners (P, role of j).  Members that join
// together (the start of a walk, a clique folded into P) are ordered by lane.
//
// Partners above the universe (the prefix) are on every path: a member's
// finished stays are summed in per-wave scratch and added to its prefix
// pairs when the wave leaves the universe, and T itself is what the
// prefix/prefix pairs are owed.  With a universe in memory these sums go to
// per-universe accumulators that a final kernel adds to the prefix pairs
// once per universe.
// Add the values of k = 2i (v0, h0) and 2i + 1 (v1, h1) of local row `row`
// to word i of the packed table: both halves with one 64-bit atomic when
// both values are below 2^32, the carries out of each half (read off the
// old word) counted in ewrap; otherwise straight to the row's u128 slots at
// out (k1_in: whether k = 2i + 1 is in the range).  Returns true if a u128
// add wrapped.
__device__ __forceinline__ bool packed_add(uint64_t *epk, uint64_t *ewrap, int kws, long long row, int i,
                                           uint64_t v0, uint64_t h0, uint64_t v1, uint64_t h1, uint64_t *out,
                                           bool k1_in) {
    if ((v0 | h0 | v1 | h1) == 0) return false;
    if (((v0 | v1) >> 32) == 0 && (h0 | h1) == 0) {
        const uint64_t x = v0 | (v1 << 32);
        const uint64_t old = atomicAdd((unsigned long long *)(epk + row * kws + i), (unsigned long long)x);
        const uint64_t c0 = ((old & 0xffffffffull) + v0) >> 32;
        const uint64_t c1 = (old + x < old) ? 1ull : 0ull;
        if (c0 | c1) atomicAdd((unsigned long long *)(ewrap + row * kws + i), (unsigned long long)(c0 | (c1 << 32)));
        return false;
    }
    bool ovf = false;
    if (v0 | h0) ovf |= atomic_add_u128(out, v0, h0);
    if (k1_in && (v1 | h1)) ovf |= atomic_add_u128(out + 2, v1, h1);
    return ovf;
}

template <int KL>
struct EdgeSink {
    // lane kk < K: running sums over the visit's leaves, types HH, HP, PP
    uint64_t t0l, t0h, t1l, t1h, t2l, t2h;
    uint64_t BH, BP;  // path members above this lane
    const int *etab;  // edge ids of the member pairs of the universe walked now
    uint64_t *xch;    // LDS hand-over slot of this wave (4 * KL words, then 64 partner lanes as bytes)
    uint64_t *snap;   // scratch [64][2][K] u128: T at the member's join (its role's two types)
    uint64_t *vacc;   // scratch [64][2][K] u128: finished stays toward hold / pivot prefix vertices
    // wave-uniform copies of the arguments
    const uint64_t *tab;
    const uint64_t *tabh;    // high limbs of the table (nullptr: every binomial used fits 64 bits)
    const uint8_t *bad;      // [bn][bn]: C(a, b) >= 2^128
    int bn;
    uint64_t *eout, *umem, *utot;
    uint64_t *epk, *ewrap;  // packed 32-bit halves (nullptr: charges go to eout)
    const int *orow, *o2e;
    int *lovf, *flags;
    int klo, K, khi, ks, ts, kw, kws;
    bool ovf;

    __device__ void init(const LevelArgs &a, uint64_t *lds_xch, int wave0) {
        xch = lds_xch;
        tab = (const uint64_t *)uniform64((uint64_t)a.bin_pad);
        tabh = (const uint64_t *)uniform64((uint64_t)a.bin_pad_hi);
        bad = (const uint8_t *)uniform64((uint64_t)a.bin_bad);
        bn = uniformi(a.bin_bn);
        eout = (uint64_t *)uniform64((uint64_t)a.vout);
        umem = (uint64_t *)uniform64((uint64_t)a.umem);
        utot = (uint64_t *)uniform64((uint64_t)a.utot);
        epk = (uint64_t *)uniform64((uint64_t)a.epk);
        ewrap = (uint64_t *)uniform64((uint64_t)a.ewrap);
        kw = uniformi(a.kw);
        kws = uniformi(a.kws);
        orow = (const int *)uniform64((uint64_t)a.orow);
        o2e = (const int *)uniform64((uint64_t)a.o2e);
        lovf = (int *)uniform64((uint64_t)a.lovf);
        flags = (int *)uniform64((uint64_t)a.flags);
        klo = uniformi(a.klo);
        K = uniformi(a.K);
        khi = klo + K - 1;
        ks = uniformi(a.kstride);
        ts = uniformi(a.tab_stride);
        const long long slot = wave0 + (long long)blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6);
        snap = a.escr + slot * (2ll * 64 * 2 * K * 2);
        snap = (uint64_t *)uniform64((uint64_t)snap);
        vacc = snap + 64 * 2 * K * 2;
        // vacc is zero on entry (cleared by the host before the first level,
        // and by every flush after use)
        ovf = false;
        BH = BP = 0;
        etab = nullptr;
        t0l = t0h = t1l = t1h = t2l = t2h = 0;
    }

    __device__ __forceinline__ void set_table(const int *t) { etab = (const int *)uniform64((uint64_t)t); }
    __device__ __forceinline__ const int *etab_ptr() const { return etab; }

    // member j (wave-uniform) joins in role P (isP) or H: record T
    __device__ __forceinline__ void snap_one(int j, bool isP, int lane) {
        if (lane < K) {
            uint64_t *d = snap + 2 * (((long long)j * 2) * K + lane);
            d[0] = isP ? t1l : t0l;
            d[1] = isP ? t1h : t0h;
            d[2 * K] = isP ? t2l : t1l;
            d[2 * K + 1] = isP ? t2h : t1h;
        }
    }

    __device__ void begin(uint64_t H, uint64_t P, int lane) {
        H = uniform64(H);
        P = uniform64(P);
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        if (((H | P) >> lane) & 1) {
            BH = H & below;
            BP = P & below;
        }
        for (uint64_t r = H | P; r; r &= r - 1) {
            const int j = __builtin_ctzll(r);
            snap_one(j, (P >> j) & 1, lane);
        }
    }

    __device__ __forceinline__ void join(int j, uint64_t Hb, uint64_t Pb, bool isP, int lane) {
        if (lane == j) {
            BH = Hb;
            BP = Pb;
        }
        snap_one(j, isP, lane);
    }

    __device__ void join_set(uint64_t Sm, uint64_t Hb, uint64_t Pb, int lane) {
        Sm = uniform64(Sm);
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        if ((Sm >> lane) & 1) {
            BH = Hb;
            BP = Pb | (Sm & below);
        }
        for (uint64_t r = Sm; r; r &= r - 1) snap_one(__builtin_ctzll(r), true, lane);
    }

    // add x (wave-uniform) to the u128 (lo, hi) of lane kk
    static __device__ __forceinline__ void add_at(uint64_t &lo, uint64_t &hi, uint64_t x, int kk, int lane) {
        const uint64_t v = (lane == kk) ? x : 0ull;
        lo += v;
        hi += (lo < v) ? 1ull : 0ull;
    }

    // the same for a 128-bit x = (xl, xh); sets ovf if the sum wraps
    __device__ __forceinline__ void add_at2(uint64_t &lo, uint64_t &hi, uint64_t xl, uint64_t xh, int kk,
                                            int lane) {
        const bool mine = lane == kk;
        const uint64_t v = mine ? xl : 0ull, u = mine ? xh : 0ull;
        lo += v;
        const uint64_t h0 = hi, c = (lo < v) ? 1ull : 0ull;
        hi = h0 + u + c;
        ovf |= hi < h0 || (hi == h0 && (u | c) != 0);
    }

    __device__ __forceinline__ void leaf(int h, int p, uint64_t, uint64_t, int lane, const LevelArgs &) {
        if (h > khi || h + p < klo) return;
        // rows of C(p, .), C(p-1, .), C(p-2, .) at column k - h, k - h - 1,
        // k - h - 2 (row -1 is all zeros and stands in for row -2: with
        // p = 0 there is no pivot vertex, so PP is never owed)
        const uint64_t *rowHH = tab + (p + 1) * ts + (klo - h + 16);
        const uint64_t *rowHP = tab + p * ts + (klo - h + 15);
        const uint64_t *rowPP = tab + max(p - 1, 0) * ts + (klo - h + 14);
        const u64x8 xHH = ldc64x8(rowHH), xHP = ldc64x8(rowHP), xPP = ldc64x8(rowPP);
        if (tabh) {
            // binomials beyond 64 bits: the high limbs from the second table
            const long long hoff = tabh - tab;
            const u64x8 yHH = ldc64x8(rowHH + hoff), yHP = ldc64x8(rowHP + hoff), yPP = ldc64x8(rowPP + hoff);
#pragma unroll
            for (int kk = 0; kk < KL; kk++) {
                if (kk < K) {
                    add_at2(t0l, t0h, xHH[kk], yHH[kk], kk, lane);
                    add_at2(t1l, t1h, xHP[kk], yHP[kk], kk, lane);
                    add_at2(t2l, t2h, xPP[kk], yPP[kk], kk, lane);
                }
            }
            // from p = 132 on a leaf may need a binomial of 2^128 or more
            if (p >= 132) {
                bool big = false;
                for (int k = klo; k <= khi; k++) {
                    for (int t = 0; t < 3; t++) {  // C(p - t, k - h - t)
                        const int r = p - t, j = k - h - t;
                        if (r >= 0 && j >= 0 && j <= r && r < bn) big |= bad[(long long)r * bn + j] != 0;
                    }
                }
                if (big && lane == 0) atomicOr(lovf, 1);
            }
            return;
        }
#pragma unroll
        for (int kk = 0; kk < KL; kk++) {
            if (kk < K) {
                add_at(t0l, t0h, xHH[kk], kk, lane);
                add_at(t1l, t1h, xHP[kk], kk, lane);
                add_at(t2l, t2h, xPP[kk], kk, lane);
            }
        }
    }

    // Word i of one pair's charges (column sel of the hand-over slots) in
    // the packed table: the values of k = 2i and 2i + 1 added to the word's
    // halves with one 64-bit atomic.  The old word gives the carries: out of
    // the low half (it went into the high half) and out of the word; both
    // are counted in ewrap and settled when the table is added to eout.  A
    // charge of 2^32 or more goes to eout itself.
    __device__ __forceinline__ void charge_word(int e, int i, int sel) {
        const int k0 = 2 * i, k1 = 2 * i + 1;
        const uint64_t v0 = xch[4 * k0 + sel], h0 = xch[4 * k0 + sel + 1];
        const uint64_t v1 = (k1 < K) ? xch[4 * k1 + sel] : 0ull, h1 = (k1 < K) ? xch[4 * k1 + sel + 1] : 0ull;
        ovf |= packed_add(epk, ewrap, kws, e, i, v0, h0, v1, h1, eout + 2 * ((long long)e * ks + k0), k1 < K);
    }

    // Member j's stay owes its partners pm (hold partners bh): every
    // (partner, word) pair is one lane's task, the words of a partner on
    // neighbouring lanes, so one instruction's atomics fall on few lines.
    __device__ __forceinline__ void charge_partners_packed(int j, uint64_t pm, uint64_t bh, int lane) {
        uint8_t *plist = (uint8_t *)(xch + 4 * KL);
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        if ((pm >> lane) & 1) plist[__popcll(pm & below)] = (uint8_t)lane;
        wave_sync();
        const int ntask = __popcll(pm) * kw;
        for (int t = lane; t < ntask; t += 64) {
            const int pi = t / kw, wi = t - pi * kw;
            const int pl = plist[pi];
            const int e = etab[j * 64 + pl];
            if (e < 0) atomicOr(flags, 4);
            else charge_word(e, wi, ((bh >> pl) & 1) ? 0 : 2);
        }
    }

    // members in L leave the path (H, P: the path they leave from)
    __device__ void leave(uint64_t L, uint64_t H, uint64_t P, int lane, int) {
        L = uniform64(L) & ((1ull << 62) - 1);
        P = uniform64(P);
        for (uint64_t rest = L; rest; rest &= rest - 1) {
            const int j = __builtin_ctzll(rest);
            const bool isP = (P >> j) & 1;
            const uint64_t bh = readlane64(BH, j), bp = readlane64(BP, j);
            // lane kk: what the stay owes toward hold (a) and pivot (b) partners
            uint64_t al = 0, ah = 0, bl = 0, bhh = 0;
            if (lane < K) {
                const uint64_t *sp = snap + 2 * (((long long)j * 2) * K + lane);
                uint64_t *va = vacc + 2 * (((long long)j * 2) * K + lane);
                const uint64_t s0l = sp[0], s0h = sp[1], s1l = sp[2 * K], s1h = sp[2 * K + 1];
                const uint64_t ta_l = isP ? t1l : t0l, ta_h = isP ? t1h : t0h;
                const uint64_t tb_l = isP ? t2l : t1l, tb_h = isP ? t2h : t1h;
                al = ta_l - s0l;
                ah = ta_h - s0h - ((ta_l < s0l) ? 1ull : 0ull);
                bl = tb_l - s1l;
                bhh = tb_h - s1h - ((tb_l < s1l) ? 1ull : 0ull);
                const uint64_t v0l = va[0], v0h = va[1], v1l = va[2 * K], v1h = va[2 * K + 1];
                const uint64_t n0 = v0l + al, n1 = v1l + bl;
                va[0] = n0;
                va[1] = v0h + ah + ((n0 < al) ? 1ull : 0ull);
                va[2 * K] = n1;
                va[2 * K + 1] = v1h + bhh + ((n1 < bl) ? 1ull : 0ull);
            }
            if ((bh | bp) == 0) continue;
            if (lane < K) {
                xch[4 * lane + 0] = al;
                xch[4 * lane + 1] = ah;
                xch[4 * lane + 2] = bl;
                xch[4 * lane + 3] = bhh;
            }
            wave_sync();
            if (epk) {
                charge_partners_packed(j, bh | bp, bh, lane);
            } else if (((bh | bp) >> lane) & 1) {
                const int e = etab[j * 64 + lane];
                if (e < 0) atomicOr(flags, 4);
                const int sel = ((bh >> lane) & 1) ? 0 : 2;
                uint64_t *dst = eout + 2 * ((long long)e * ks);
                for (int kk = 0; kk < K; kk++) {
                    const uint64_t l = xch[4 * kk + sel], hv = xch[4 * kk + sel + 1];
                    if (e >= 0 && (l | hv)) ovf |= atomic_add_u128(dst + 2 * kk, l, hv);
                }
            }
            wave_sync();
        }
    }

    // The wave leaves the universe (every stay of a member is finished):
    // prefix pairs.  With root >= 0 the prefix is that single hold vertex;
    // otherwise the sums go to universe `uni`'s accumulators.
    __device__ void flush(int lane, int nm, int, int root, int2, int uni, const LevelArgs &) {
        root = uniformi(root);
        uni = uniformi(uni);
        nm = uniformi(nm);
        if (root >= 0) {
            // a light root's walk: member `lane` is the root's lane-th out-neighbour
            if (lane < nm) {
                const int e = o2e[orow[root] + lane];
                if (e < 0) atomicOr(flags, 4);
                const uint64_t *va = vacc + 2 * (((long long)lane * 2) * K);
                for (int kk = 0; kk < K; kk++) {
                    const uint64_t l = va[2 * kk], hv = va[2 * kk + 1];
                    if (e >= 0 && (l | hv)) ovf |= atomic_add_u128(eout + 2 * ((long long)e * ks + kk), l, hv);
                }
            }
        } else if (uni >= 0) {
            if (lane < nm) {
                const uint64_t *va = vacc + 2 * (((long long)lane * 2) * K);
                uint64_t *um = umem + 2 * ((((long long)uni * 64 + lane) * 2) * K);
                for (int i = 0; i < 2 * K; i++) {
                    const uint64_t l = va[2 * i], hv = va[2 * i + 1];
                    if (l | hv) ovf |= atomic_add_u128(um + 2 * i, l, hv);
                }
            }
            if (lane < K) {
                uint64_t *ut = utot + 2 * ((long long)uni * 3 * K + lane);
                if (t0l | t0h) ovf |= atomic_add_u128(ut, t0l, t0h);
                if (t1l | t1h) ovf |= atomic_add_u128(ut + 2 * K, t1l, t1h);
                if (t2l | t2h) ovf |= atomic_add_u128(ut + 4 * K, t2l, t2h);
            }
        }
        if (ovf) atomicOr(lovf, 1);
        ovf = false;
        if (lane < nm) {
            uint64_t *va = vacc + 2 * (((long long)lane * 2) * K);
            for (int i = 0; i < 4 * K; i++) va[i] = 0ull;
        }
        t0l = t0h = t1l = t1h = t2l = t2h = 0;
    }
};

template <int KL, int LK>
struct SinkOf {
    using T = VertexSink<KL, LK == PV_LK_VERTEX128>;
};
template <int KL>
struct SinkOf<KL, PV_LK_EDGE> {
    using T = EdgeSink<KL>;
};

// Work counters of a wave: SCT nodes visited; pivot work, the sum over
// nodes of |S| * ceil(|S|/64) (64-bit AND+popcount pairs); and the extra
// words of multi-word children, the sum over nodes with |S| > 64 of
// (children) * (ceil(|S|/64) - 1).  Every other child is formed with one
// word operation, so the child work, the sum over internal nodes of
// (children) * ceil(|S|/64), is (nodes - roots) + extra.
struct Ctr {
    unsigned long long nodes, work, child;
};

// Phase timing (built with -DPV_PHASE_TIMING only): wall time per phase of
// a wave's units, summed over waves, in 10 ns ticks of s_memrealtime.
#ifdef PV_PHASE_TIMING
#define PT_N 16
// sub-phase sums of compact walks, per wave in LDS: [0] lane batches, [1]
// leaf read-off of the wave tier, [2] lane-batch loop trips, [3] nodes the
// lanes of those batches visited
__device__ __forceinline__ unsigned long long *pt_sub() {
    __shared__ unsigned long long s_pt_sub[WAVES_PER_BLOCK][4];
    return s_pt_sub[threadIdx.x >> 6];
}
#define PT_MARK(t) const uint64_t t = __builtin_amdgcn_s_memrealtime()
#define PT_ADD(slot, t0) (pt[slot] += __builtin_amdgcn_s_memrealtime() - (t0))
#else
#define PT_MARK(t)
#define PT_ADD(slot, t0)
#endif

template <int KL, int LK>
__device__ int make_universe(uint64_t A, int nm, int gid, int lane, const LevelArgs &a,
                             int root, int grp, uint64_t Hw, uint64_t Pw, const int *vl, int W,
                             int2 &pref, const int *src_etab);

// ------------------------------------------------------------ lane tier
// On sparse graphs most SCT nodes have a set of at most 8 vertices, and a
// wave that walks such a node keeps most of its lanes idle.  The compact
// walk instead queues these nodes, one per lane, and walks up to 64 of
// their subtrees at once, each lane its own: the induced adjacency of the
// node's set as eight 8-bit rows in one register (local index = rank in
// the universe, so "smallest id" is still "lowest bit"), and the depth-first
// stack of at most 7 frames (a frame's set strictly contains the next one's
// and has at least 2 vertices) in LDS, frame t of lane l at [t][l] (no bank
// conflicts).  Pivot rule, child order and the node, work and leaf
// accounting are those of compact_dfs: same tree, same counts.

__device__ __forceinline__ uint64_t shfl64(uint64_t x, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)x, src, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(x >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t row8(uint64_t rows, int i) {
    return (uint32_t)(rows >> (8 * i)) & 0xFFu;
}

// LDS slots of the lane tier's per-member sums (per vertex): member j's
// slot kk of this wave at [j * (KL + 1) + kk]; zero between batches
template <int KL>
__device__ __forceinline__ lds_u64 *lane_acc() {
    __shared__ unsigned long long s_lacc[WAVES_PER_BLOCK][64 * (KL + 1)];
    return (lds_u64 *)s_lacc[threadIdx.x >> 6];
}

// the lane tier's depth-first frames of this wave: frame t of lane l at
// [t][l]; at most PV_LANE_MAX - 1 frames (each needs |S| >= 2, sets shrink)
__device__ __forceinline__ uint32_t (*lane_frames())[64] {
    __shared__ uint32_t s_lst[WAVES_PER_BLOCK][PV_LANE_MAX - 1][64];
    return s_lst[threadIdx.x >> 6];
}

// Walk the queued subtrees: lane i < qn holds node qS (a set of at most
// PV_LANE_MAX members of the universe whose row for member `lane` is A) with
// path totals h = qhp & 0xFFFF, p = qhp >> 16.  For per-vertex counts, bit i
// of a member lane's qmH (qmP) says that the member was a hold (pivot)
// vertex of the i-th queued node's path; lanes 62 and 63 stand for the hold
// and pivot vertices above the universe, as in VertexSink.  All lanes take
// part.
//
// Per-vertex counts (Alg. 2): a leaf owes C(p, k-h) to every hold vertex of
// its path and C(p-1, k-h-1) to every pivot vertex.  Members taken inside
// the lane's subtree get theirs at the leaf through LDS atomics on their
// slots.  For the vertices above a queued node every leaf of its subtree
// owes the same, so the lane sums its leaves' binomials; a member is on the
// path for runs of consecutive queued nodes, and a run [a, b) owes the
// difference of two inclusive prefix sums of those sums over the lanes.
template <int KL, bool LOC, class VS>
__device__ __forceinline__ void lane_walk(uint64_t A, uint64_t qS, uint64_t qmH, uint64_t qmP, uint32_t qhp,
                                          int qn, int lane, int hlim, GlobalSink &gs, VS &vs,
                                          uint32_t &nodes, uint32_t &work, uint32_t &nleaves) {
    constexpr int NK = LOC ? KL : 1;
    const bool act = lane < qn;
    const uint64_t S0 = act ? qS : 0ull;
    const int s = __popcll(S0);
    // members in increasing order (6 bits each in mpack) and their rows
    // restricted to S0, as 8-bit local masks (byte i = row of the i-th member)
    int m[PV_LANE_MAX];
    uint64_t T = S0, mpack = 0;
#pragma unroll
    for (int i = 0; i < PV_LANE_MAX; i++) {
        m[i] = T ? __builtin_ctzll(T) : 0;
        mpack |= (uint64_t)m[i] << (6 * i);
        T &= T - 1ull;  // stays 0 once empty
    }
    const uint32_t smask = (1u << s) - 1u;
    uint64_t rows = 0;
#pragma unroll
    for (int i = 0; i < PV_LANE_MAX; i++) {
        const uint64_t r = shfl64(A, m[i]);
        uint32_t b = 0;
#pragma unroll
        for (int j = 0; j < PV_LANE_MAX; j++) b |= (uint32_t)((r >> m[j]) & 1ull) << j;
        if (i >= s) b = 0;
        rows |= (uint64_t)(b & smask) << (8 * i);
    }
    const int h0 = (int)(qhp & 0xFFFFu), p0 = (int)(qhp >> 16);
    uint32_t S = smask;
    uint32_t Hl = 0, Pl = 0;  // hold / pivot members taken inside the subtree (local masks)
    int depth = 0;
    uint32_t(*st)[64] = lane_frames();
    lds_u64 *acc = nullptr;
    if constexpr (LOC) {
        acc = lane_acc<KL>();
        vs.park(acc + lane * (KL + 1));
        wave_sync();
    }
    uint64_t sH[NK], sP[NK];  // this lane's sums toward the vertices above its node
#pragma unroll
    for (int kk = 0; kk < NK; kk++) sH[kk] = sP[kk] = 0;
    uint32_t nn = 0, ww = 0, nl = 0;
    bool visit = true, live = act;
#ifdef PV_PHASE_TIMING
    uint32_t trips = 0;
#endif
    while (live) {
#ifdef PV_PHASE_TIMING
        trips++;
#endif
        if (visit) {
            nn++;
            if (S != 0 && h0 + __popc(Hl) < hlim) {
                const int sc = __popc(S);
                ww += (uint32_t)sc;
                int best = -1, piv = 0;
                bool full = true;
#pragma unroll
                for (int i = 0; i < PV_LANE_MAX; i++) {
                    if ((S >> i) & 1u) {
                        const int c = __popc(row8(rows, i) & S);
                        if (c > best) {
                            best = c;
                            piv = i;
                        }
                        full = full && (c + 1 == sc);
                    }
                }
                PV_ASSERT(gs.chk_flags, gs.chk_line, ((S >> piv) & 1u) && (Hl & Pl) == 0 && (S & (Hl | Pl)) == 0);
                if (best + 1 != sc) {
                    // frame: set, pivot, path members; then the pivot child
                    PV_ASSERT(gs.chk_flags, gs.chk_line, depth < PV_LANE_MAX - 1);
                    st[depth][lane] = S | ((uint32_t)piv << 8) | (Hl << 11) | (Pl << 19);
                    depth++;
                    S &= row8(rows, piv);
                    Pl |= 1u << piv;
                    continue;
                }
                if (!full) {
                    // the pivot sees all of S: no hold child
                    S &= ~(1u << piv);
                    Pl |= 1u << piv;
                    continue;
                }
                // S is a clique: its pivot chain ends in one leaf
                nn += (uint32_t)sc;
                ww += (uint32_t)(sc * (sc - 1) / 2);
                Pl |= S;
            }
            nl++;
            const int h = h0 + __popc(Hl), p = p0 + __popc(Pl);
            gs.leaf_lane(h, p);
            if (LOC && h <= vs.khi && h + p >= vs.klo) {
                // same table segments as VertexSink::leaf
                const uint64_t *rowH = vs.tab + (p + 1) * vs.ts + (vs.klo - h + 16);  // C(p, k-h)
                const uint64_t *rowP = vs.tab + p * vs.ts + (vs.klo - h + 15);        // C(p-1, k-h-1)
                uint64_t vH[NK], vP[NK];
#pragma unroll
                for (int kk = 0; kk < NK; kk++) {
                    vH[kk] = rowH[kk];
                    vP[kk] = rowP[kk];
                    sH[kk] += vH[kk];
                    sP[kk] += vP[kk];
                }
                for (uint32_t M = Hl | Pl; M; M &= M - 1u) {
                    const int i = __builtin_ctz(M);
                    const bool isH = (Hl >> i) & 1u;
                    lds_u64 *slot = acc + (int)((mpack >> (6 * i)) & 63u) * (KL + 1);
#pragma unroll
                    for (int kk = 0; kk < NK; kk++)
                        __hip_atomic_fetch_add(slot + kk, isH ? vH[kk] : vP[kk], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
        }
        visit = true;
        if (depth == 0) {
            live = false;
            continue;
        }
        // next hold child of the top frame
        const int t = depth - 1;
        const uint32_t F = st[t][lane];
        const uint32_t Sf = F & 0xFFu;
        const int pf = (int)((F >> 8) & 7u);
        const uint32_t R = Sf & ~row8(rows, pf) & ~(1u << pf);
        const int v = __builtin_ctz(R);
        S = row8(rows, v) & Sf;
        if ((R & (R - 1u)) == 0) depth--;
        else st[t][lane] = F & ~(1u << v);
        Hl = ((F >> 11) & 0xFFu) | (1u << v);
        Pl = (F >> 19) & 0xFFu;
    }
#ifdef PV_PHASE_TIMING
    {
        // the wave ran as many trips as its longest lane
        const uint32_t tmax = wave_max_u32(trips);
        const uint32_t tot = wave_sum_u32(nn);
        if (lane == 0) {
            pt_sub()[2] += tmax;
            pt_sub()[3] += tot;
        }
    }
#endif
    nodes += wave_sum_u32(nn);
    work += wave_sum_u32(ww);
    nleaves += wave_sum_u32(nl);
    if constexpr (LOC) {
        // members taken inside the subtrees: their LDS slots (then cleared)
        wave_sync();
        vs.add_slots(acc + lane * (KL + 1), lane);
        wave_sync();
        // the vertices above the queued nodes.  The slot region (64 x
        // (KL + 1) entries, free again) holds rows [v][lane] of 8 values
        // (4 k-slots x hold / pivot); lane v < 8 turns row v into its
        // inclusive prefix sums over the first qn lanes, and a member adds,
        // for each of its runs [a, b), entry b-1 minus entry a-1
        static_assert(KL + 1 >= 8, "slot region too small for the distribution");
        const int qn8 = (qn + 7) & ~7;
#pragma unroll
        for (int k0 = 0; k0 < NK; k0 += 4) {
#pragma unroll
            for (int v = 0; v < 8; v++) {
                const int kk = k0 + (v >> 1);
                acc[v * 64 + lane] = (kk < NK) ? ((v & 1) ? sP[kk] : sH[kk]) : 0ull;
            }
            wave_sync();
            if (lane < 8) {
                lds_u64 *row = acc + lane * 64;
                uint64_t run = 0;
#pragma unroll 1
                for (int L0 = 0; L0 < qn8; L0 += 8) {
                    uint64_t x[8];
#pragma unroll
                    for (int i = 0; i < 8; i++) x[i] = row[L0 + i];
#pragma unroll
                    for (int i = 0; i < 8; i++) {
                        run += x[i];
                        row[L0 + i] = run;
                    }
                }
            }
            wave_sync();
            uint64_t add[8];
#pragma unroll
            for (int v = 0; v < 8; v++) add[v] = 0;
#pragma unroll
            for (int role = 0; role < 2; role++) {
                for (uint64_t M = role ? qmP : qmH; M;) {
                    const int a0 = __builtin_ctzll(M);
                    const uint64_t Z = ~M & (~0ull << a0);
                    const int b0 = Z ? __builtin_ctzll(Z) : 64;
                    M = (b0 == 64) ? 0ull : (M & (~0ull << b0));
#pragma unroll
                    for (int v = role; v < 8; v += 2)
                        add[v] += acc[v * 64 + b0 - 1] - (a0 > 0 ? acc[v * 64 + a0 - 1] : 0ull);
                }
            }
#pragma unroll
            for (int v = 0; v < 8; v++) {
                const int kk = k0 + (v >> 1);
                if (kk < NK) vs.add_val(kk, add[v]);
            }
            wave_sync();
        }
        // the region starts the next batch at zero
        for (int i = lane; i < 8 * 64; i += 64) acc[i] = 0ull;
        wave_sync();
    }
}

// ------------------------------------------------ work queues
// Units handed from one wave to others: compact node and frame items, and
// multi-word items.  Level by level (persist = 0) a producer appends to the
// next level's array and the kernel boundary makes the items visible.  In
// the persistent walk the compact queue is split into PV_QSLICES slices
// (a wave pushes to its home slice, so the reservation atomics of different
// waves spread over eight cache lines), every slot has a flag that the
// producer sets after its item is written and released, and consumers claim
// slots with a compare-and-swap on the slice's head.

__device__ __forceinline__ int home_slice() {
    return (int)(((blockIdx.x * blockDim.x + threadIdx.x) >> 6) % PV_QSLICES);
}

__device__ __forceinline__ int ld_agent(const unsigned long long *p) {
    return (int)(uint32_t)__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// the call's abort flag (cancellation or the host's watchdog)
__device__ __forceinline__ int call_aborted(const LevelArgs &a) {
    return a.abort ? __hip_atomic_load(a.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
}

// Reserve n consecutive slots for this wave's items in the queue whose
// reservation counter is *tail (capacity cap; in the persistent walk rdy
// are its slot flags, base its first slot).  Returns the first slot (an
// index into the item array) or -1 when they do not fit: the overflow flag
// is set, and the host walks the tree again with larger buffers.  Reserved
// slots inside the array are then marked never-written (a consumer skips
// them) and those past its end count as done at once, so the walk still
// ends.  Wave-uniform; every lane of the wave takes part.
__device__ int reserve_slots(const LevelArgs &a, int *tail, int *rdy, int base, int cap, int n, int lane) {
    int t = 0;
    if (lane == 0) t = atomicAdd(tail, n);
    t = bcast0(t);
    if (t + n <= cap) return base + t;
    if (a.persist) {
        for (int i = t + lane; i < min(t + n, cap); i += 64)
            __hip_atomic_store(&rdy[base + i], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (lane == 0)
            atomicAdd(&a.pctl->done.v, (unsigned long long)(t + n - max(t, cap)));
    }
    if (lane == 0) atomicOr(a.flags, 1);
    return -1;
}

__device__ __forceinline__ int reserve_items(const LevelArgs &a, int n, int lane) {
    if (!a.persist) return reserve_slots(a, a.c_out_n, nullptr, 0, a.c_cap, n, lane);
    const int s = home_slice();
    return reserve_slots(a, (int *)&a.pctl->ctail[s].v, a.cready, s * a.c_scap, a.c_scap, n, lane);
}

__device__ __forceinline__ int reserve_mw_items(const LevelArgs &a, int n, int lane) {
    if (!a.persist) return reserve_slots(a, a.mw_out_n, nullptr, 0, a.mw_cap, n, lane);
    return reserve_slots(a, (int *)&a.pctl->mtail.v, a.mready, 0, a.m_cap, n, lane);
}

// The items of slots [first, first + n) are written: release them (a fence
// over all of this wave's stores), then set their flags.  Every lane of the
// wave takes part.
__device__ __forceinline__ void publish_slots(const LevelArgs &a, int *rdy, int first, int n, int lane) {
    if (!a.persist) return;
    __threadfence();
    for (int i = lane; i < n; i += 64)
        __hip_atomic_store(&rdy[first + i], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Claim one slot of a queue (head/tail lines of nsl slices of cap slots,
// slice s0 first): its index into the item array, or -1 if every slice is
// drained for now.  Wave-uniform.
__device__ int claim_slot(PvLine *head, PvLine *tail, int nsl, int cap, int s0, int lane) {
    int got = -1;
    if (lane == 0) {
        for (int i = 0; i < nsl && got < 0; i++) {
            const int sl = (s0 + i) % nsl;
            int h = ld_agent(&head[sl].v);
            const int t = min(ld_agent(&tail[sl].v), cap);
            while (h < t) {
                const int prev = atomicCAS((int *)&head[sl].v, h, h + 1);
                if (prev == h) {
                    got = sl * cap + h;
                    break;
                }
                h = prev;
            }
        }
    }
    return bcast0(got);
}

// Wait until the producer of a claimed slot has published it: 1 written,
// 2 never written (its reservation did not fit); 0 after a bounded wait
// (error bit 2 set).  The acquire fence makes the item's words visible to
// every lane.
__device__ int wait_slot(const LevelArgs &a, const int *rdy, int lane) {
    int r = 0;
    if (lane == 0) {
        for (uint32_t spins = 0;; spins++) {
            r = __hip_atomic_load(rdy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (r) break;
            if (spins > (1u << 22)) {
                atomicOr((int *)&a.pctl->state.v, 2);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    r = bcast0(r);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return r;
}

// ------------------------------------------------------ compact-tier DFS
// Walk the whole subtree of node (S, H, P, h, p) of a compact universe
// whose row for member `lane` is A.  Depth first, stack in lane-indexed
// registers (frame t in lane t; at most 63 frames since every frame's set
// is a strict superset of the next one's).

// After dfs_budget visited nodes the walk stops and hands the rest of its
// subtree to the next level: the node it was about to visit becomes a node
// item and every frame on its stack a frame item (the frame's remaining set,
// pivot and path), which the receiving wave resumes by walking that frame's
// remaining hold children.  The universe is written out first if it only
// lived in registers.  So no single wave walks an unbounded subtree, and a
// split hands over depth + 1 items however wide the frames are.
template <int KL, int LK, bool LT = true>
__device__ void compact_dfs(uint64_t A, uint64_t S, uint64_t H, uint64_t P, int h, int p, int lane,
                            const LevelArgs &a, GlobalSink &gs, typename SinkOf<KL, LK>::T &vs,
                            Ctr &ct, int &uni, int nm, int gid, int root, bool from_frame,
                            uint32_t fmeta) {
    constexpr bool EDGE = LK == PV_LK_EDGE;
    constexpr bool LOCAL = KL > 0;
    uint64_t stS = 0, stH = 0, stP = 0;
    uint32_t stM = 0;
    int depth = 0;
    S = uniform64(S);
    H = uniform64(H);
    P = uniform64(P);
    h = uniformi(h);
    p = uniformi(p);
    if (LOCAL) vs.begin(H, P, lane);
    // per-call counters: a call visits at most dfs_budget + 128 <= 2^20 + 128
    // nodes and adds at most 2080 work per node, so 32 bits suffice
    uint32_t nodes = 0, work = 0, nleaves = 0;
    const int kmax = uniformi(a.kmax);
    // a hold child (h + 1 holds) exists only while h < hlim
    const int hlim = kmax > 0 ? kmax : 0x7fffffff;
    const uint32_t limit = (uint32_t)uniformi(a.dfs_budget);
    // lane tier (global counts; per vertex with 64-bit sums and 8 k-slots):
    // nodes with |S| <= lmax are queued, lane qn holding the qn-th, and
    // walked 64 at a time.  LT = false compiles it out (a kernel whose walks
    // are too small to fill a batch keeps its registers for occupancy).
    constexpr bool LANE = LT && (!LOCAL || (LK == PV_LK_VERTEX64 && KL == 8));
    const int lmax = LANE ? uniformi(a.lane_max) : 0;
    uint64_t qS = 0, qmH = 0, qmP = 0;
    uint32_t qhp = 0;
    int qn = 0;
    bool visit = true;
    if (uniformi(from_frame ? 1 : 0)) {
        // resume an unfinished frame: only its remaining hold children are
        // left (S is the frame's set with the visited ones removed)
        stS = writelane64(stS, S, 0);
        if (LOCAL) {
            stH = writelane64(stH, H, 0);
            stP = writelane64(stP, P, 0);
        }
        stM = writelane32(stM, uniform32(fmeta), 0);
        depth = 1;
        visit = false;
    }
    for (;;) {
        bool queued = false;
        if constexpr (LANE) {
            if (visit && S != 0 && h < hlim && __popcll(S) <= lmax) {
                if (lane == qn) {
                    qS = S;
                    qhp = (uint32_t)h | ((uint32_t)p << 16);
                }
                if (LOCAL) {
                    // this member's role on the queued node's path (lanes
                    // 62/63: the vertices above the universe)
                    const bool inH = ((H >> lane) & 1) || lane == 62;
                    const bool inP = !inH && (((P >> lane) & 1) || lane == 63);
                    qmH |= (uint64_t)inH << qn;
                    qmP |= (uint64_t)inP << qn;
                }
                if (++qn == 64) {
#ifdef PV_PHASE_TIMING
                    const uint64_t t_lw = __builtin_amdgcn_s_memrealtime();
#endif
                    lane_walk<KL, LOCAL>(A, qS, qmH, qmP, qhp, qn, lane, hlim, gs, vs, nodes, work, nleaves);
#ifdef PV_PHASE_TIMING
                    if (lane == 0) pt_sub()[0] += __builtin_amdgcn_s_memrealtime() - t_lw;
#endif
                    qn = 0;
                    qmH = qmP = 0;
                }
                queued = true;
            }
        }
        if (visit && !queued) {
            nodes++;
            // with h = k_max hold vertices (truncated tree) the rest of the
            // subtree is one pivot chain whose single leaf counts only toward
            // C_{k_max} (C(p', 0) = 1 for any p'), as a leaf here does
            if (S != 0 && h < hlim) {
                const int s = __popcll(S);
                work += (uint32_t)s;
                const bool in = (S >> lane) & 1;
                const uint32_t c = (uint32_t)__popcll(A & S);
                const uint32_t key = in ? (((c + 1u) << 6) | (uint32_t)(63 - lane)) : 0u;
                const uint32_t best = wave_max_u32(key);
                const int piv = 63 - (int)(best & 63u);
                const int pc = (int)(best >> 6) - 1;
                const uint64_t pbit = 1ull << piv;
                PV_ASSERT(a.flags, a.check, ((S >> piv) & 1) && (nm <= 0 || nm >= 64 || (S >> nm) == 0));
                PV_ASSERT(a.flags, a.check, !LOCAL || ((H & P) == 0 && (S & (H | P)) == 0));
                if (pc + 1 == s) {
                    // the pivot sees all of S: no hold child.  If every member
                    // does, S is a clique and its pivot chain ends in one leaf.
                    if (ballot64(in && (int)c + 1 != s) == 0) {
                        nodes += (uint32_t)s;
                        work += (uint32_t)(s * (s - 1) / 2);
                        if (LOCAL) {
                            vs.join_set(S, H, P, lane);
                            P |= S;
                        }
                        p += s;
                    } else {
                        S &= ~pbit;
                        if (LOCAL) {
                            vs.join(piv, H, P, true, lane);
                            P |= pbit;
                        }
                        p++;
                        continue;
                    }
                } else {
                    const uint64_t Ap = readlane64(A, piv);
                    if (h < hlim) {
                        PV_ASSERT(a.flags, a.check, depth < 64);
                        // frame `depth` in lane `depth` (one lane index for the four writes)
                        const bool at = lane_id_here() == depth;
                        stS = at ? S : stS;
                        if (LOCAL) {
                            stH = at ? H : stH;
                            stP = at ? P : stP;
                        }
                        stM = at ? ((uint32_t)piv | ((uint32_t)h << 6) | ((uint32_t)p << 19)) : stM;
                        depth++;
                    }
                    S &= Ap;
                    if (LOCAL) {
                        vs.join(piv, H, P, true, lane);
                        P |= pbit;
                    }
                    p++;
                    continue;
                }
            }
            // a leaf: S is empty (or a clique folded into P above)
            nleaves++;
#ifdef PV_PHASE_TIMING
            const uint64_t t_lf = __builtin_amdgcn_s_memrealtime();
#endif
            gs.leaf(h, p, lane);
            if (LOCAL) vs.leaf(h, p, H, P, lane, a);
#ifdef PV_PHASE_TIMING
            if (lane == 0) pt_sub()[1] += __builtin_amdgcn_s_memrealtime() - t_lf;
#endif
        }
        visit = true;
        if (depth == 0) break;
        // next hold child of the top frame
        const int t = depth - 1;
        const uint64_t Sf = readlane64(stS, t);
        const uint32_t M = readlane32(stM, t);
        const int pf = (int)(M & 63u);
        const uint64_t R = Sf & ~readlane64(A, pf) & ~(1ull << pf);
        const int v = __builtin_ctzll(R);
        const uint64_t vbit = 1ull << v;
        S = readlane64(A, v) & Sf;
        if ((R & (R - 1)) == 0) depth--;
        else stS = writelane64(stS, Sf & ~vbit, t);
        h = (int)((M >> 6) & 0x1FFFu) + 1;
        p = (int)(M >> 19);
        if (LOCAL) {
            const uint64_t Ht = readlane64(stH, t), Pt = readlane64(stP, t);
            vs.leave((H | P) & ~(Ht | Pt), H, P, lane, gid);
            vs.join(v, Ht, Pt, false, lane);
            H = Ht | vbit;
            P = Pt;
        }
        // budget spent: the pending hold child and every stack frame become
        // items of the next level (checked where a walk resumes a frame, so a
        // call visits at most dfs_budget plus one pivot chain)
        if (nodes >= limit && depth > 0) {
            if (uni < 0) {
                int2 pref;
                uni = make_universe<KL, LK>(A, nm, gid, lane, a, root, -1, 0ull, 0ull, nullptr, 0, pref,
                                              EDGE ? vs.etab_ptr() : nullptr);
                if (uni < 0) break;  // buffers full: the host reruns with larger ones
            }
            const int total = depth + 1;
            const int slot = reserve_items(a, total, lane);
            if (slot < 0) break;
            CItem it;
            if (lane == 0) {
                it.S = S;
                it.H = H;
                it.P = P;
                it.uni = (uint32_t)uni;
                it.hp = (uint32_t)h | ((uint32_t)p << 16);
                a.c_out[slot] = it;
            }
            if (lane < depth) {  // lane t holds frame t
                it.S = stS;
                it.H = LOCAL ? stH : 0ull;
                it.P = LOCAL ? stP : 0ull;
                it.uni = (uint32_t)uni | 0x80000000u;
                it.hp = stM;
                a.c_out[slot + 1 + lane] = it;
            }
            publish_slots(a, a.cready, slot, total, lane);
            break;
        }
    }
    if constexpr (LANE) {
        if (qn > 0) {
#ifdef PV_PHASE_TIMING
            const uint64_t t_lw = __builtin_amdgcn_s_memrealtime();
#endif
            lane_walk<KL, LOCAL>(A, qS, qmH, qmP, qhp, qn, lane, hlim, gs, vs, nodes, work, nleaves);
#ifdef PV_PHASE_TIMING
            if (lane == 0) pt_sub()[0] += __builtin_amdgcn_s_memrealtime() - t_lw;
#endif
        }
    }
    if (LOCAL) vs.leave(H | P, H, P, lane, gid);
    ct.nodes += nodes;
    ct.work += work;
    gs.add_leaves(nleaves, lane);
}

// ---------------------------------------------------- compact-tier chain
// Follow the pivot chain of node (S,H,P,h,p) in universe `uni`; hold
// children go to the next level; once |S| <= dfs_max finish depth first.
// root/pref name the vertices above the universe (local counts only).

template <int KL, int LK, bool LT = true>
__device__ void compact_run(uint64_t A, uint64_t S, uint64_t H, uint64_t P, int h, int p, int uni,
                            int nm, int gid, int root, int2 pref, int lane, const LevelArgs &a,
                            GlobalSink &gs, typename SinkOf<KL, LK>::T &vs, Ctr &ct,
                            bool from_frame = false, uint32_t fmeta = 0) {
    constexpr bool EDGE = LK == PV_LK_EDGE;
    constexpr bool LOCAL = KL > 0;
    S = uniform64(S);
    H = uniform64(H);
    P = uniform64(P);
    h = uniformi(h);
    p = uniformi(p);
    uni = uniformi(uni);
    nm = uniformi(nm);
#ifdef PV_CHECKED
    {
        // the universe's adjacency: rows inside the members, no loops,
        // symmetric.  Walks of global counts do not carry the member count
        // (nm = 0): then every lane is checked (a non-member's row is empty).
        const int nmc = (nm > 0 && nm < 64) ? nm : 64;
        const bool mem = lane < nmc;
        bool okA = !mem || (((A >> lane) & 1) == 0 && (nmc >= 64 || (A >> nmc) == 0));
        for (int j = 0; j < nmc; j++) {
            const uint64_t Aj = readlane64(A, j);
            okA = okA && (!mem || ((Aj >> lane) & 1) == ((A >> j) & 1));
        }
        PV_ASSERT(a.flags, a.check, okA && (nmc >= 64 || (S >> nmc) == 0));
    }
#endif
    // truncated tree: at h = k_max the subtree is one leaf (see compact_dfs);
    // a frame item carries its path totals in fmeta, not in h and p
    if (!from_frame && a.kmax > 0 && h >= a.kmax) S = 0;
    for (;;) {
        const int s = __popcll(S);
        if (from_frame || s <= a.dfs_max || uni < 0) {
            compact_dfs<KL, LK, LT>(A, S, H, P, h, p, lane, a, gs, vs, ct, uni, nm, gid, root,
                                  from_frame, fmeta);
            break;
        }
        ct.nodes++;
        ct.work += (unsigned long long)s;
        const bool in = (S >> lane) & 1;
        const uint32_t c = (uint32_t)__popcll(A & S);
        const uint32_t key = in ? (((c + 1u) << 6) | (uint32_t)(63 - lane)) : 0u;
        const uint32_t best = wave_max_u32(key);
        const int piv = 63 - (int)(best & 63u);
        const int pc = (int)(best >> 6) - 1;
        const uint64_t pbit = 1ull << piv;
        if (pc + 1 == s) {
            if (ballot64(in && (int)c + 1 != s) == 0) {
                ct.nodes += (unsigned long long)s;
                ct.work += (unsigned long long)s * (unsigned long long)(s - 1) / 2;
                if (LOCAL) {
                    vs.begin(H, P, lane);
                    vs.join_set(S, H, P, lane);
                    P |= S;
                }
                p += s;
                gs.leaf(h, p, lane);
                gs.add_leaves(1, lane);
                if (LOCAL) {
                    vs.leaf(h, p, H, P, lane, a);
                    vs.leave(H | P, H, P, lane, gid);
                }
                break;
            }
            S &= ~pbit;
            if (LOCAL) P |= pbit;
            p++;
            continue;
        }
        const uint64_t Ap = readlane64(A, piv);
        const uint64_t R = S & ~Ap & ~pbit;
        if (!(a.kmax > 0 && h + 1 > a.kmax)) {
            // hold child of member v (v in R, increasing): N(S,v) minus the
            // earlier non-neighbours; lane v builds its own child
            const int nR = __popcll(R);
            const int slot = reserve_items(a, nR, lane);
            if (slot >= 0) {
                if ((R >> lane) & 1) {
                    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
                    CItem it;
                    it.S = A & S & ~(R & below);
                    it.H = H | (1ull << lane);
                    it.P = P;
                    it.uni = (uint32_t)uni;
                    it.hp = (uint32_t)(h + 1) | ((uint32_t)p << 16);
                    a.c_out[slot + __popcll(R & below)] = it;
                }
                publish_slots(a, a.cready, slot, nR, lane);
            }
        }
        S &= Ap;
        if (LOCAL) P |= pbit;
        p++;
    }
    // the caller flushes the per-vertex accumulators (vs.flush) when it
    // leaves this universe
}

// Write a compact universe (rows, member ids, prefix list); returns its
// index or -1 when the buffers are full.  For per-edge counts it also
// clears the universe's prefix-pair accumulators (each lane the slots it
// adds to later).
template <int KL, int LK>
__device__ int make_universe(uint64_t A, int nm, int gid, int lane, const LevelArgs &a,
                             int root, int grp, uint64_t Hw, uint64_t Pw, const int *vl, int W,
                             int2 &pref, const int *src_etab) {
    constexpr bool EDGE = LK == PV_LK_EDGE;
    constexpr bool LOCAL = KL > 0;
    int uni = 0;
    if (lane == 0) uni = atomicAdd(a.u_n, 1);
    uni = bcast0(uni);
    if (uni >= a.u_cap) {
        if (lane == 0) atomicOr(a.flags, 1);
        return -1;
    }
    a.u_rows[(long long)uni * 64 + lane] = (lane < nm) ? A : 0ull;
    if (a.vgraph && lane == 0) a.u_root[uni] = root;  // batch: names the universe's graph
    if (LOCAL && !EDGE && lane == 0) a.u_grp[uni] = grp;
    pref = make_int2(0, 0);
    if (LOCAL) {
        a.u_gid[(long long)uni * 64 + lane] = (lane < nm) ? gid : -1;
        // prefix: the root plus the hold and pivot vertices above (word-major
        // multi-word sets Hw/Pw, lane w = word w)
        const int nh = (lane < W) ? __popcll(Hw) : 0, np = (lane < W) ? __popcll(Pw) : 0;
        const int tot = (int)wave_sum_u32((uint32_t)(nh + np)) + 1;
        int off = 0;
        if (lane == 0) off = atomicAdd(a.pref_n, tot);
        off = bcast0(off);
        if (off + tot > a.pref_cap) {
            if (lane == 0) atomicOr(a.flags, 1);
        } else {
            if (lane == 0) a.pref_pool[off] = root;
            int cur = off + 1;
            for (int w = 0; w < W; w++) {
                const uint64_t hw = readlane64(Hw, w), pw = readlane64(Pw, w);
                const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
                // per vertex: local indices (grouped by heavy root later); per edge: ids
                const int x = EDGE ? vl[w * 64 + lane] : w * 64 + lane;
                if ((hw >> lane) & 1) a.pref_pool[cur + __popcll(hw & below)] = x;
                cur += __popcll(hw);
                if ((pw >> lane) & 1) a.pref_pool[cur + __popcll(pw & below)] = (int)((unsigned)x | 0x80000000u);
                cur += __popcll(pw);
            }
            pref = make_int2(off, tot);
            if (lane == 0) a.u_pref[uni] = pref;
        }
        if (!EDGE && lane < a.K) {
            // per-vertex: the universe's totals owed to its prefix, hold and pivot
            uint64_t *ut = a.utot + 2 * ((long long)uni * 2 * a.K + lane);
            ut[0] = ut[1] = 0ull;
            ut[2 * a.K] = ut[2 * a.K + 1] = 0ull;
        }
        if (EDGE) {
            const int K = a.K;
            uint64_t *um = a.umem + 2 * (((long long)uni * 64 + lane) * 2 * K);
            for (int i = 0; i < 4 * K; i++) um[i] = 0ull;
            // prefix/prefix sums: HH and HP from lane 62, PP from lane 63
            uint64_t *ut = a.utot + 2 * ((long long)uni * 3 * K);
            if (lane == 62)
                for (int i = 0; i < 4 * K; i++) ut[i] = 0ull;
            if (lane == 63)
                for (int i = 0; i < 2 * K; i++) ut[4 * K + i] = 0ull;
            // edge ids of the member pairs: copied from the walk's own table,
            // or looked up once here (u_gid above must be visible first)
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
            __builtin_amdgcn_wave_barrier();
            int *dst = a.ueid + (long long)uni * 4096;
            if (src_etab) {
                for (int r = 0; r < nm; r++) dst[r * 64 + lane] = src_etab[r * 64 + lane];
            } else if (lane < nm) {
                const uint64_t above = (lane == 63) ? 0ull : (~0ull << (lane + 1));
                uint64_t rest = A & above;
                while (rest) {
                    const int j = __builtin_ctzll(rest);
                    rest &= rest - 1;
                    const int gj = a.u_gid[(long long)uni * 64 + j];
                    const int e = edge_id(gid, gj, a.sub, a.orow, a.ocol, a.o2e);
                    dst[lane * 64 + j] = e;
                    dst[j * 64 + lane] = e;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
            __builtin_amdgcn_wave_barrier();
        }
    }
    return uni;
}

// ---------------------------------------------------- multi-word tier
// Node sets over a heavy universe of up to 64*W vertices, lane w holding
// word w.  Rows are word-major in HBM: row u, word w at rows[w*dpad + u].

// Word w of member u's row: from HBM (stride dpad) or from a copy staged in
// LDS for the unit (same layout).
struct RowsG {
    const uint64_t *p;
    int stride;
    __device__ __forceinline__ uint64_t operator()(int w, int u) const { return p[(long long)w * stride + u]; }
};
struct RowsL {
    const lds_u64 *p;
    int stride;
    __device__ __forceinline__ uint64_t operator()(int w, int u) const { return p[w * stride + u]; }
};

// Returns true with a compact start state (A, S0, nm, gid, uni, root,
// pref, h, p) once |S| <= 64, false if the buffers were full.
struct CState {
    uint64_t A, S, H, P;
    int h, p, uni, nm, gid, root;
    int2 pref;
#ifdef PV_PHASE_TIMING
    uint64_t t_re;  // time of the re-index into a compact universe
#endif
};

template <int KL, int LK, class R>
__device__ bool mw_run(R rows, int hu, uint64_t Sw, uint64_t Hw, uint64_t Pw, int h, int p, int lane,
                       const LevelArgs &a, Ctr &ct, int *memb, CState &cs) {
    constexpr bool EDGE = LK == PV_LK_EDGE;
    constexpr bool LOCAL = KL > 0;
    const int W = a.W, dpad = a.dpad;
    const int *vl = a.hu_vl + (long long)hu * dpad;
    const int root = a.order[a.heavy_base + hu];
    const bool wl = lane < W;
    if (!wl) Sw = Hw = Pw = 0;
    // truncated tree: at h = k_max the subtree is one leaf (see compact_dfs)
    if (a.kmax > 0 && h >= a.kmax) Sw = 0;
    for (;;) {
        const int s = (int)wave_sum_u32(wl ? (uint32_t)__popcll(Sw) : 0u);
        if (s <= PV_LIGHT_MAX) {
#ifdef PV_PHASE_TIMING
            const uint64_t t_r = __builtin_amdgcn_s_memrealtime();
#endif
            // re-index S into a compact universe (members in id order)
            int base = 0;
            for (int t = 0; t < W; t++) {
                const uint64_t St = readlane64(Sw, t);
                const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
                if ((St >> lane) & 1) memb[base + __popcll(St & below)] = t * 64 + lane;
                base += __popcll(St);
            }
            wave_sync();
            const int mj = (lane < s) ? memb[lane] : 0;
            wave_sync();
            // member lane's row over the members (bit c: member c, in id
            // order): its row words, all read at once, each compressed to
            // the members of that word
            uint64_t rw[4];
#pragma unroll
            for (int t = 0; t < 4; t++) rw[t] = (t < W && lane < s) ? rows(t, mj) : 0ull;
            uint64_t A = 0;
            int c0 = 0;
            for (int t = 0; t < W; t++) {
                const uint64_t St = readlane64(Sw, t);
                const uint64_t r = (t < 4) ? (t == 0 ? rw[0] : t == 1 ? rw[1] : t == 2 ? rw[2] : rw[3])
                                           : ((lane < s) ? rows(t, mj) : 0ull);
                int c = c0;
                for (uint64_t m = St; m; m &= m - 1, c++) A |= ((r >> __builtin_ctzll(m)) & 1ull) << c;
                c0 = c;
            }
            const int gid = (lane < s) ? vl[mj] : -1;
            int2 pref = make_int2(0, 0);
            int uni = -1;
            // the root and the multi-word holds/pivots form the prefix
            if (s > a.dfs_max || LOCAL) {
                uni = make_universe<KL, LK>(A, s, gid, lane, a, root, a.heavy_base + hu, Hw, Pw, vl, W, pref, nullptr);
                if (uni < 0) return false;  // buffers full: the host reruns with larger ones
            }
            cs.A = A;
            cs.S = (s == 64) ? ~0ull : ((1ull << s) - 1);
            cs.H = cs.P = 0;
            cs.h = h;
            cs.p = p;
            cs.uni = uni;
            cs.nm = s;
            cs.gid = gid;
            cs.root = -1;
            cs.pref = pref;
#ifdef PV_PHASE_TIMING
            cs.t_re = __builtin_amdgcn_s_memrealtime() - t_r;
#endif
            return true;
        }
        ct.nodes++;
        ct.work += (unsigned long long)s * (unsigned long long)((s + 63) / 64);
        // pivot: argmax over u in S of |N(S,u)|, ties to the smallest index
        uint32_t best = 0;
        for (int t = 0; t < W; t++) {
            const uint64_t St = readlane64(Sw, t);
            const int u = t * 64 + lane;
            if ((St >> lane) & 1) {
                uint32_t c = 0;
                for (int w = 0; w < W; w++) c += (uint32_t)__popcll(rows(w, u) & readlane64(Sw, w));
                best = max(best, ((c + 1u) << 12) | (uint32_t)(4095 - u));
            }
        }
        best = wave_max_u32(best);
        const int piv = 4095 - (int)(best & 4095u);
        const int pc = (int)(best >> 12) - 1;
        const int pw = piv >> 6;
        PV_ASSERT(a.flags, a.check, pw < W && ((readlane64(Sw, pw) >> (piv & 63)) & 1) && pc >= 0 && pc < s);
        const uint64_t pb = (lane == pw) ? (1ull << (piv & 63)) : 0ull;
        const uint64_t Ap = wl ? rows(lane, piv) : 0ull;
        {
            // the pivot child and the hold children are formed word by word
            const bool holds = pc + 1 != s && !(a.kmax > 0 && h + 1 > a.kmax);
            ct.child += (unsigned long long)(holds ? s - pc : 1) * (unsigned long long)((s + 63) / 64 - 1);
        }
        if (pc + 1 != s && !(a.kmax > 0 && h + 1 > a.kmax)) {
            // hold children, increasing id, each N(S,v) minus earlier ones
            uint64_t Rw = Sw & ~Ap & ~pb;
            uint64_t Scur = Sw;
            const int nR = (int)wave_sum_u32(wl ? (uint32_t)__popcll(Rw) : 0u);
            const int slot = reserve_mw_items(a, nR, lane);
            if (slot >= 0) {
                for (int i = 0; i < nR; i++) {
                    const uint64_t nzw = ballot64(wl && Rw != 0);
                    const int w0 = __builtin_ctzll(nzw);
                    const int v = w0 * 64 + __builtin_ctzll(readlane64(Rw, w0));
                    const uint64_t vb = (lane == w0) ? (1ull << (v & 63)) : 0ull;
                    uint64_t *it = a.mw_out + (long long)(slot + i) * a.mw_stride;
                    if (wl) {
                        it[lane] = rows(lane, v) & Scur;
                        it[W + lane] = Hw | vb;
                        it[2 * W + lane] = Pw;
                    }
                    if (lane == 0)
                        it[3 * W] = (uint64_t)(uint32_t)hu |
                                    ((uint64_t)((uint32_t)(h + 1) | ((uint32_t)p << 16)) << 32);
                    Scur &= ~vb;
                    Rw &= ~vb;
                }
                publish_slots(a, a.mready, slot, nR, lane);
            }
        }
        // continue with the pivot child N(S, piv)
        Sw &= Ap;
        Pw |= pb;
        p++;
    }
}

// ------------------------------------------------------ gathers of roots
// Induced adjacency of N+(v): for each u_j in N+(v) and each w in N+(u_j),
// w in N+(v) at position i means u_j ~ u_i (each edge inside N+(v) is seen
// once, from its smaller-key end).
//
// A light root's members' out-lists are flattened over the lanes, 64 edges
// a step.  The owner of edge q is the member with the largest start <= q
// among those with a nonempty list: a wave-wide OR marks the starts that
// fall in the step, and a popcount below the lane ranks the owner.  Whether
// the other end w is a member, and which, comes from a hash of the member
// ids in LDS (HS slots, linear probing, at most 62 keys).  The kernels of
// global counts, whose occupancy the LDS bounds, take 128 slots; the
// per-vertex and per-edge kernels, bound by registers, take 256 (shorter
// probe runs).

template <int HS>
__device__ __forceinline__ int gather_slot(int x) {
    static_assert(HS == 128 || HS == 256, "hash of 7 or 8 bits");
    return (int)(((uint32_t)x * 2654435761u) >> (HS == 256 ? 24 : 25));
}

template <int HS>
__device__ uint64_t gather_light(int v, int lane, const LevelArgs &a, int *s_nz, int *s_base,
                                 unsigned long long *s_A, int *s_hk, uint8_t *s_hv, int &d, int &gid, int *etab) {
    const int b = a.orow[v];
    d = a.orow[v + 1] - b;
    const int u = (lane < d) ? a.ocol[b + lane] : 0x7fffffff;
    gid = (lane < d) ? u : -1;
    const int ub = (lane < d) ? a.orow[u] : 0;
    const int od = (lane < d) ? (a.orow[u + 1] - ub) : 0;
    const int incl = wave_incl_scan(od);
    const int total = (int)readlane32((uint32_t)incl, 63);
    const int pre = incl - od;  // this member's first edge in the flattened order
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint64_t nzm = ballot64(od > 0);
    if (od > 0) s_nz[__popcll(nzm & below)] = lane;  // rank among nonempty lists -> member
    // edge q of the flattened lists sits at ocol[s_base[j] + q] (member j
    // owning q): no second read of the row pointers
    s_base[lane] = ub - pre;
    s_A[lane] = 0ull;
#pragma unroll
    for (int i = 0; i < HS / 64; i++) s_hk[lane + 64 * i] = -1;
    wave_sync();
    if (lane < d) {
        int h = gather_slot<HS>(u);
        while (atomicCAS(&s_hk[h], -1, u) != -1) h = (h + 1) & (HS - 1);
        s_hv[h] = (uint8_t)lane;
    }
    wave_sync();
    for (int q0 = 0; q0 < total; q0 += 64) {
        // starts of nonempty lists in [q0, q0 + 64), and how many came before
        const bool inwin = od > 0 && pre >= q0 && pre < q0 + 64;
        const int sh = inwin ? pre - q0 : 0;
        const uint32_t mlo = wave_or_u32((inwin && sh < 32) ? 1u << sh : 0u);
        const uint32_t mhi = wave_or_u32((inwin && sh >= 32) ? 1u << (sh - 32) : 0u);
        const uint64_t mwin = ((uint64_t)mhi << 32) | mlo;
        const int before = __popcll(ballot64(od > 0 && pre < q0));
        const int q = q0 + lane;
        if (q < total) {
            const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
            const int j = s_nz[before + __popcll(mwin & upto) - 1];
            const int pos = s_base[j] + q;
            const int w = a.ocol[pos];
            int h = gather_slot<HS>(w), l2 = -1;
            for (;;) {
                const int k = s_hk[h];
                if (k == w) {
                    l2 = s_hv[h];
                    break;
                }
                if (k < 0) break;
                h = (h + 1) & (HS - 1);
            }
            if (l2 >= 0) {
                atomicOr(&s_A[j], 1ull << l2);
                atomicOr(&s_A[l2], 1ull << j);
                if (etab) {
                    // per-edge counts: the pair's edge id comes with the oriented edge
                    const int e = a.o2e[pos];
                    etab[j * 64 + l2] = e;
                    etab[l2 * 64 + j] = e;
                }
            }
        }
    }
    if (etab) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
        __builtin_amdgcn_wave_barrier();
    }
    wave_sync();
    const uint64_t A = (lane < d) ? (uint64_t)s_A[lane] : 0ull;
    wave_sync();
    return A;
}

__device__ void gather_heavy(int hu, int v, int lane, const LevelArgs &a) {
    const int W = a.W, dpad = a.dpad;
    uint64_t *rows = a.hu_rows + (long long)hu * W * dpad;
    int *vl = a.hu_vl + (long long)hu * dpad;
    const int b = a.orow[v];
    const int d = a.orow[v + 1] - b;
    for (int j = lane; j < dpad; j += 64) vl[j] = (j < d) ? a.ocol[b + j] : 0x7fffffff;
    for (long long i = lane; i < (long long)W * dpad; i += 64) rows[i] = 0ull;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
    __builtin_amdgcn_wave_barrier();
    for (int j = 0; j < d; j++) {
        const int uj = vl[j];
        const int e0 = a.orow[uj], e1 = a.orow[uj + 1];
        for (int e = e0 + lane; e < e1; e += 64) {
            const int w = a.ocol[e];
            int lo = 0, hi = d;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (vl[mid] < w) lo = mid + 1; else hi = mid;
            }
            if (lo < d && vl[lo] == w) {
                atomicOr((unsigned long long *)&rows[(long long)(lo >> 6) * dpad + j],
                         1ull << (lo & 63));
                atomicOr((unsigned long long *)&rows[(long long)(j >> 6) * dpad + lo],
                         1ull << (j & 63));
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
    __builtin_amdgcn_wave_barrier();
}

// The same gather with the universe built in LDS (W <= 3): rows at
// lrows[w * dpad + u] (the HBM layout), member ids in lvl.  The members'
// out-lists are flattened: lane q of a pass takes edge q of their
// concatenation, finds its owner j by binary search over the exclusive
// prefix of the out-degrees (held in registers, member j in lane j % 64,
// slot j / 64) and the other end among the members by binary search in
// LDS, and sets the pair's two bits with LDS atomics.  The rows and ids are
// then copied to HBM for the universe's units at later levels.
__device__ __forceinline__ int slot_of(int v0, int v1, int v2, int m) {
    const int src = m & 63;
    const int a0 = __shfl(v0, src, 64), a1 = __shfl(v1, src, 64), a2 = __shfl(v2, src, 64);
    const int sl = m >> 6;
    return sl == 0 ? a0 : (sl == 1 ? a1 : a2);
}

__device__ void gather_heavy_lds(int hu, int v, int lane, const LevelArgs &a, lds_u64 *lrows, int *lvl) {
    const int W = a.W, dpad = a.dpad;
    uint64_t *rows = a.hu_rows + (long long)hu * W * dpad;
    int *vl = a.hu_vl + (long long)hu * dpad;
    const int b = a.orow[v];
    const int d = a.orow[v + 1] - b;  // <= dpad <= 192
    int id[3], st[3], ln[3];
#pragma unroll
    for (int t = 0; t < 3; t++) {
        const int j = t * 64 + lane;
        id[t] = (j < d) ? a.ocol[b + j] : 0x7fffffff;
    }
#pragma unroll
    for (int t = 0; t < 3; t++) {
        const int j = t * 64 + lane;
        st[t] = (j < d) ? a.orow[id[t]] : 0;
        ln[t] = (j < d) ? a.orow[id[t] + 1] - st[t] : 0;
        if (j < dpad) lvl[j] = id[t];
    }
    for (int i = lane; i < W * dpad; i += 64) lrows[i] = 0ull;
    // exclusive prefix of the out-degrees over the members, and each
    // member's base: edge q of member j sits at ocol[base_j + q]
    int off[3], base[3];
    int run = 0;
#pragma unroll
    for (int t = 0; t < 3; t++) {
        const int incl = wave_incl_scan(ln[t]);
        off[t] = run + incl - ln[t];
        base[t] = st[t] - off[t];
        run += (int)readlane32((uint32_t)incl, 63);
    }
    const int total = run;
    wave_sync();
    for (int q0 = 0; q0 < total; q0 += 64) {
        const int q = q0 + lane;
        // owner: the last member j < d with off_j <= q (uniform trip count)
        int j = 0;
#pragma unroll
        for (int step = 128; step > 0; step >>= 1) {
            const int m = j + step;
            const int om = slot_of(off[0], off[1], off[2], min(m, d - 1));
            if (m < d && om <= q) j = m;
        }
        const int bj = slot_of(base[0], base[1], base[2], j);
        if (q < total) {
            const int w = a.ocol[bj + q];
            // w's position among the members: how many ids are below it
            int pos = 0;
#pragma unroll
            for (int step = 128; step > 0; step >>= 1)
                if (pos + step <= d && lvl[pos + step - 1] < w) pos += step;
            if (pos < d && lvl[pos] == w) {
                __hip_atomic_fetch_or(lrows + (pos >> 6) * dpad + j, 1ull << (pos & 63), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_fetch_or(lrows + (j >> 6) * dpad + pos, 1ull << (j & 63), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
    wave_sync();
    for (int i = lane; i < W * dpad; i += 64) rows[i] = lrows[i];
    for (int i = lane; i < dpad; i += 64) vl[i] = lvl[i];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
    __builtin_amdgcn_wave_barrier();
}

// --------------------------------------------------------- level kernel
// One launch per unit kind and level, each with its own register budget:
//   PV_UNITS_MW     multi-word items of the previous level, and at level 0
//                   the heavy roots (gather + multi-word chain)
//   PV_UNITS_ITEMS  compact items of the previous level (the bulk of the tree)
//   PV_UNITS_LIGHT  level 0 only: roots with |N+(v)| <= PV_LIGHT_MAX,
//                   gathered into registers (largest first)
// Every wave takes units from the launch's own cursor until none is left.

// Units of a kind are claimed a chunk at a time, one atomic per chunk: a
// single cursor taken by every wave one unit at a time serialises across the
// XCDs (about 14 ns per claim, which bounded a launch over a million small
// roots).  Chunks interleave: chunk c holds units c, c + nch, c + 2 nch, ...
// of the first n0 units, so units that sit next to each other in a queue
// (the pieces of one split subtree, roots of equal degree) go to different
// waves; the units from n0 on (8 per wave of the launch) are claimed one at
// a time, so waves finish together.  The host picks n0 and nch.  All values
// wave-uniform; -1 when the kind's n units are gone.
// A claim that takes a new chunk also reads the call's abort flag (set by
// the host to cancel, or by its watchdog): once it is set, no unit is
// handed out, so every wave finishes the unit in hand and exits.
struct Claim {
    int idx = -1;
    __device__ __forceinline__ int next(int *cursor, int n, int n0, int nch, int lane, const int *abort) {
        if (idx >= 0) {
            idx += nch;
            if (idx < n0) return idx;
        }
        int b = 0, stop = 0;
        if (lane == 0) {
            b = atomicAdd(cursor, 1);
            if (abort) stop = __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (bcast0(__shfl(stop, 0, 64))) {
            idx = -1;
            return -1;
        }
        const int c = bcast0(__shfl(b, 0, 64));
        if (c < nch) {
            idx = c;
            return idx;
        }
        idx = -1;
        const int t = n0 + (c - nch);
        return t < n ? t : -1;
    }
    // the next call returns a unit of the chunk in hand without an atomic
    __device__ __forceinline__ bool mid_chunk(int n0, int nch) const { return idx >= 0 && idx + nch < n0; }
};

// The per-vertex kernels with 64-bit visit sums (the lane tier's member
// slots in LDS) are held to 128 VGPRs and 16 LDS histogram rows, so that
// four waves share a SIMD: the walk is bound by the latency of each node's
// dependent steps, and the fourth wave hides more of it than the registers
// spilled to scratch cost.
template <int KL, int LK, int MODE>
struct LevelShape {
    static constexpr bool V64 = KL == 8 && LK == PV_LK_VERTEX64;
    // (the persistent walk keeps the budget of the compact-item kernel, whose
    // units are the bulk of its work).  The light-root kernel has no lane
    // tier and fits five waves without spills (per vertex, 1M-vertex graph:
    // its launch 6.6 -> 5.3 ms); the other per-vertex kinds spill at five
    // (step 44.7 -> 51.3 ms).
    static constexpr int waves_per_simd = V64 ? (MODE == PV_UNITS_LIGHT ? 5 : 4) : 3;
    static constexpr int lds_h = V64 ? 16 : PV_LDS_H;
};

template <int KL, int MODE, int LK>
__global__ void __launch_bounds__(64 * WAVES_PER_BLOCK, (LevelShape<KL, LK, MODE>::waves_per_simd))
    sct_level_kernel(const LevelArgs *__restrict__ pa) {
    constexpr bool EDGE = LK == PV_LK_EDGE;
    constexpr bool LOCAL = KL > 0;
    constexpr int LDS_H = LevelShape<KL, LK, MODE>::lds_h;
    const LevelArgs &a = *pa;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    __shared__ unsigned long long s_bins[LDS_H * 64];
    for (int i = threadIdx.x; i < LDS_H * 64; i += blockDim.x) s_bins[i] = 0ull;
    __syncthreads();
    GlobalSink gs;
    gs.init(a, s_bins, LDS_H);
    typename SinkOf<KL, LK>::T vs;
    __shared__ uint64_t s_xch[WAVES_PER_BLOCK][EDGE ? 4 * KL + 8 : 1];
    if (LOCAL) vs.init(a, s_xch[wv], EDGE ? a.escr_wave0[MODE] : 0);
    if constexpr (LOCAL && LK == PV_LK_VERTEX64 && KL == 8 && MODE != PV_UNITS_LIGHT) {
        // the lane tier's per-member slots of this wave start at zero
        lds_u64 *acc = lane_acc<KL>();
        for (int i = lane; i < 64 * (KL + 1); i += 64) acc[i] = 0ull;
        wave_sync();
    }
    Ctr ct;
    ct.nodes = ct.work = ct.child = 0;
#ifdef PV_PHASE_TIMING
    uint64_t pt[PT_N];
    for (int i = 0; i < PT_N; i++) pt[i] = 0;
    if (lane == 0) pt_sub()[0] = pt_sub()[1] = pt_sub()[2] = pt_sub()[3] = 0ull;
    PT_MARK(pt_kernel0);
#endif
    constexpr int CK = MODE == PV_UNITS_ALL ? PV_UNITS_LIGHT : MODE;  // the claim cursor of a static range
    int *cursor = a.next + CK;
    const int claim_n0 = uniformi(a.n0[CK]), claim_nch = uniformi(a.nch[CK]);
    Claim claim;
    // persistent walk: pivot work per unit kind
    unsigned long long wk[3] = {0ull, 0ull, 0ull};

    if constexpr (MODE == PV_UNITS_MW) {
        __shared__ int s_memb[WAVES_PER_BLOCK][64];
        const int n0 = a.n_mw_in, n1 = n0 + (a.level == 0 ? a.nheavy : 0);
        for (;;) {
            const int idx = claim.next(cursor, n1, claim_n0, claim_nch, lane, a.abort);
            if (idx < 0) break;
            int hu, h = 1, p = 0;
            uint64_t Sw = 0, Hw = 0, Pw = 0;
            // the universe's rows staged in LDS for the unit (per vertex with
            // 64-bit sums, W <= 3): in the lane tier's slots, which the
            // walk below needs only after the multi-word part and which
            // are cleared again before it
            constexpr bool STAGE = LOCAL && LK == PV_LK_VERTEX64 && KL == 8;
            const bool staged = STAGE && a.W <= 3 && a.W * a.dpad <= 64 * (KL + 1);
            lds_u64 *lrows = STAGE ? lane_acc<KL>() : nullptr;
            if (idx < n0) {
                const uint64_t *it = a.mw_in + (long long)idx * a.mw_stride;
                const bool wl = lane < a.W;
                Sw = wl ? it[lane] : 0ull;
                Hw = wl ? it[a.W + lane] : 0ull;
                Pw = wl ? it[2 * a.W + lane] : 0ull;
                const uint64_t meta = it[3 * a.W];
                hu = (int)(uint32_t)meta;
                const uint32_t hp = (uint32_t)(meta >> 32);
                h = (int)(hp & 0xFFFFu);
                p = (int)(hp >> 16);
                if (staged) {
                    const uint64_t *src = a.hu_rows + (long long)uniformi(hu) * a.W * a.dpad;
                    for (int i = lane; i < a.W * a.dpad; i += 64) lrows[i] = src[i];
                    wave_sync();
                }
            } else {
                hu = idx - n0;
                const int v = a.order[a.heavy_base + hu];
                PT_MARK(t_g);
                if (staged) gather_heavy_lds(hu, v, lane, a, lrows, (int *)lane_frames());
                else gather_heavy(hu, v, lane, a);
                PT_ADD(0, t_g);
                const int d = a.orow[v + 1] - a.orow[v];
                // root node N+(v): every member; the root is the first hold vertex
                if (lane < a.W) {
                    const int cnt = min(max(d - lane * 64, 0), 64);
                    Sw = (cnt == 64) ? ~0ull : ((1ull << cnt) - 1);
                }
            }
            gs.set_vertex(a.order[a.heavy_base + hu]);
            CState cs;
            PT_MARK(t_m);
            bool ok;
            if (staged) {
                ok = mw_run<KL, LK>(RowsL{lrows, a.dpad}, hu, Sw, Hw, Pw, h, p, lane, a, ct, s_memb[wv], cs);
                // the lane tier's slots start at zero
                wave_sync();
                for (int i = lane; i < a.W * a.dpad; i += 64) lrows[i] = 0ull;
                wave_sync();
            } else {
                ok = mw_run<KL, LK>(RowsG{a.hu_rows + (long long)uniformi(hu) * a.W * a.dpad, a.dpad}, hu, Sw, Hw,
                                    Pw, h, p, lane, a, ct, s_memb[wv], cs);
            }
            PT_ADD(1, t_m);
#ifdef PV_PHASE_TIMING
            if (ok) pt[10] += cs.t_re;
#endif
            if (ok) {
                if (EDGE) vs.set_table(a.ueid + (long long)cs.uni * 4096);
                PT_MARK(t_c);
                compact_run<KL, LK>(cs.A, cs.S, cs.H, cs.P, cs.h, cs.p, cs.uni, cs.nm, cs.gid, cs.root,
                                cs.pref, lane, a, gs, vs, ct);
                PT_ADD(2, t_c);
                PT_MARK(t_f);
                if (LOCAL) vs.flush(lane, cs.nm, cs.gid, cs.root, cs.pref, cs.uni, a);
                PT_ADD(3, t_f);
            }
        }
    } else if constexpr (MODE == PV_UNITS_ITEMS) {
        const int n = a.n_c_in;
        for (;;) {
            const int idx = claim.next(cursor, n, claim_n0, claim_nch, lane, a.abort);
            if (idx < 0) break;
            PT_MARK(t_l);
            const CItem it = a.c_in[idx];
            const uint32_t uw = uniform32(it.uni);
            const int u = (int)(uw & 0x7fffffffu);
            const bool fr = (uw >> 31) != 0;
            const uint64_t A = a.u_rows[(long long)u * 64 + lane];
            if (a.vgraph) gs.set_vertex(a.u_root[u]);
            int gid = -1;
            int2 pref = make_int2(0, 0);
            if (LOCAL) {
                gid = a.u_gid[(long long)u * 64 + lane];
                pref = a.u_pref[u];
            }
            const int nm = (int)wave_sum_u32(gid >= 0 ? 1u : 0u);
            if (EDGE) vs.set_table(a.ueid + (long long)u * 4096);
            PT_ADD(4, t_l);
            PT_MARK(t_c);
            compact_run<KL, LK>(A, it.S, it.H, it.P, (int)(it.hp & 0xFFFFu), (int)(it.hp >> 16), u, nm,
                            gid, -1, pref, lane, a, gs, vs, ct, fr, it.hp);
            PT_ADD(5, t_c);
            PT_MARK(t_f);
            if (LOCAL) vs.flush(lane, nm, gid, -1, pref, u, a);
            PT_ADD(6, t_f);
        }
    } else if constexpr (MODE == PV_UNITS_ALL) {
        // The persistent walk: units in order of preference -- multi-word
        // items, heavy roots, compact items, light roots -- until every unit
        // is done.  A wave counts the units it finished and adds them to the
        // shared count when it finds nothing to take; the walk is over once
        // that count equals the roots plus every reserved queue slot (read in
        // that order: a unit's pushes precede its count, so the sum cannot
        // meet the count while work is left).
        __shared__ int s_memb[WAVES_PER_BLOCK][64];
        __shared__ int s_nz[WAVES_PER_BLOCK][64];
        __shared__ int s_base[WAVES_PER_BLOCK][64];
        __shared__ unsigned long long s_A[WAVES_PER_BLOCK][64];
        constexpr int GATHER_HS = LOCAL ? 256 : 128;
        __shared__ int s_hk[WAVES_PER_BLOCK][GATHER_HS];
        __shared__ uint8_t s_hv[WAVES_PER_BLOCK][GATHER_HS];
        int *etab_w = EDGE ? a.weid + (long long)(blockIdx.x * WAVES_PER_BLOCK + wv) * 4096 : nullptr;
        PersistCtl *pc = (PersistCtl *)uniform64((uint64_t)a.pctl);
        const int home = home_slice();
        const int nheavy = uniformi(a.nheavy), nlight = uniformi(a.nlight);
        const int c_scap = uniformi(a.c_scap), m_cap = uniformi(a.m_cap);
        const unsigned long long nroots = (unsigned long long)nheavy + (unsigned long long)nlight;
        bool heavy_left = nheavy > 0, light_left = nlight > 0;
        uint32_t my_done = 0, since_check = 0;
        unsigned long long seen_done = ~0ull;
        uint64_t t_seen = 0;
        for (;;) {
            // abort or error: checked every 16 units and whenever idle
            if (++since_check >= 16) {
                since_check = 0;
                if (bcast0(ld_agent(&pc->state.v) | ld_agent(&pc->abort.v) | call_aborted(a))) break;
            }
            const unsigned long long w0 = ct.work;
            int kind = -1;
            if (light_left && claim.mid_chunk(claim_n0, claim_nch)) {
                kind = PV_UNITS_LIGHT;
            } else {
                // multi-word items, then heavy roots
                int slot = claim_slot(&pc->mhead, &pc->mtail, 1, m_cap, 0, lane);
                int hu = -1;
                if (slot < 0 && heavy_left) {
                    int b = 0;
                    if (lane == 0) b = atomicAdd(a.next + PV_UNITS_MW, 1);
                    b = bcast0(b);
                    if (b < nheavy) hu = b;
                    else heavy_left = false;
                }
                if (slot >= 0 || hu >= 0) {
                    kind = PV_UNITS_MW;
                    int h = 1, p = 0;
                    uint64_t Sw = 0, Hw = 0, Pw = 0;
                    bool skip = false;
                    if (slot >= 0) {
                        const int r = wait_slot(a, a.mready + slot, lane);
                        if (r != 1) {
                            skip = true;
                        } else {
                            const uint64_t *it = a.mw_out + (long long)slot * a.mw_stride;
                            const bool wl = lane < a.W;
                            Sw = wl ? it[lane] : 0ull;
                            Hw = wl ? it[a.W + lane] : 0ull;
                            Pw = wl ? it[2 * a.W + lane] : 0ull;
                            const uint64_t meta = it[3 * a.W];
                            hu = uniformi((int)(uint32_t)meta);
                            const uint32_t hp = uniform32((uint32_t)(meta >> 32));
                            h = (int)(hp & 0xFFFFu);
                            p = (int)(hp >> 16);
                        }
                    } else {
                        const int v = a.order[a.heavy_base + hu];
                        gather_heavy(hu, v, lane, a);
                        const int d = a.orow[v + 1] - a.orow[v];
                        if (lane < a.W) {
                            const int cnt = min(max(d - lane * 64, 0), 64);
                            Sw = (cnt == 64) ? ~0ull : ((1ull << cnt) - 1);
                        }
                    }
                    if (!skip) {
                        gs.set_vertex(a.order[a.heavy_base + hu]);
                        CState cs;
                        if (mw_run<KL, LK>(RowsG{a.hu_rows + (long long)hu * a.W * a.dpad, a.dpad}, hu, Sw, Hw, Pw, h,
                                           p, lane, a, ct, s_memb[wv], cs)) {
                            if (EDGE) vs.set_table(a.ueid + (long long)cs.uni * 4096);
                            compact_run<KL, LK>(cs.A, cs.S, cs.H, cs.P, cs.h, cs.p, cs.uni, cs.nm, cs.gid, cs.root,
                                                cs.pref, lane, a, gs, vs, ct);
                            if (LOCAL) vs.flush(lane, cs.nm, cs.gid, cs.root, cs.pref, cs.uni, a);
                        }
                    }
                } else {
                    // compact node and frame items
                    slot = claim_slot(pc->chead, pc->ctail, PV_QSLICES, c_scap, home, lane);
                    if (slot >= 0) {
                        kind = PV_UNITS_ITEMS;
                        if (wait_slot(a, a.cready + slot, lane) == 1) {
                            const CItem it = a.c_out[slot];
                            const uint32_t uw = uniform32(it.uni);
                            const int u = (int)(uw & 0x7fffffffu);
                            const bool fr = (uw >> 31) != 0;
                            const uint64_t A = a.u_rows[(long long)u * 64 + lane];
                            if (a.vgraph) gs.set_vertex(a.u_root[u]);
                            int gid = -1;
                            int2 pref = make_int2(0, 0);
                            if (LOCAL) {
                                gid = a.u_gid[(long long)u * 64 + lane];
                                pref = a.u_pref[u];
                            }
                            const int nm = (int)wave_sum_u32(gid >= 0 ? 1u : 0u);
                            if (EDGE) vs.set_table(a.ueid + (long long)u * 4096);
                            compact_run<KL, LK>(A, it.S, it.H, it.P, (int)(it.hp & 0xFFFFu), (int)(it.hp >> 16), u,
                                                nm, gid, -1, pref, lane, a, gs, vs, ct, fr, it.hp);
                            if (LOCAL) vs.flush(lane, nm, gid, -1, pref, u, a);
                        }
                    } else if (light_left) {
                        kind = PV_UNITS_LIGHT;
                    }
                }
            }
            if (kind == PV_UNITS_LIGHT) {
                const int idx = claim.next(cursor, nlight, claim_n0, claim_nch, lane, a.abort);
                if (idx < 0) {
                    light_left = false;
                    kind = -1;
                } else {
                    const int v = a.order[a.light_base + idx];
                    gs.set_vertex(v);
                    if (EDGE) vs.set_table(etab_w);
                    int d, gid;
                    const uint64_t A = gather_light<GATHER_HS>(v, lane, a, s_nz[wv], s_base[wv], s_A[wv], s_hk[wv], s_hv[wv], d,
                                                    gid, etab_w);
                    int uni = -1;
                    int2 pref = make_int2(0, 0);
                    bool ok = true;
                    if (d > a.dfs_max) {
                        uni = make_universe<KL, LK>(A, d, gid, lane, a, v, -1, 0ull, 0ull, nullptr, 0, pref, etab_w);
                        ok = uni >= 0;  // buffers full: the host walks again with larger ones
                    }
                    if (ok) {
                        const int root = (uni < 0) ? v : -1;
                        compact_run<KL, LK, false>(A, (d == 64) ? ~0ull : ((1ull << d) - 1), 0ull, 0ull, 1, 0, uni, d,
                                                   gid, root, pref, lane, a, gs, vs, ct);
                        if (LOCAL) vs.flush(lane, d, gid, root, pref, uni, a);
                    }
                }
            }
            if (kind >= 0) {
                my_done++;
                wk[kind] += ct.work - w0;
                // hand the count in now and then, so that idle waves see progress
                if (my_done >= 256) {
                    if (lane == 0) atomicAdd(&pc->done.v, (unsigned long long)my_done);
                    my_done = 0;
                }
                continue;
            }
            // nothing to take now: hand in the finished count, then see
            // whether the walk is over
            if (lane == 0 && my_done) atomicAdd(&pc->done.v, (unsigned long long)my_done);
            my_done = 0;
            unsigned long long D = 0, T = 0;
            int bad = 0;
            if (lane == 0) {
                D = __hip_atomic_load(&pc->done.v, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                T = nroots + (unsigned long long)(uint32_t)ld_agent(&pc->mtail.v);
                for (int sl = 0; sl < PV_QSLICES; sl++) T += (unsigned long long)(uint32_t)ld_agent(&pc->ctail[sl].v);
                bad = ld_agent(&pc->state.v) | ld_agent(&pc->abort.v) | call_aborted(a);
            }
            D = uniform64(D);
            T = uniform64(T);
            if (D >= T || bcast0(bad)) break;
            // no unit finished or queued anywhere for 10 s (s_memrealtime
            // counts at 100 MHz; a unit walks at most dfs_budget nodes): give
            // up with an error instead of waiting for ever
            const uint64_t now = __builtin_amdgcn_s_memrealtime();
            if (D + (T << 32) != seen_done) {
                seen_done = D + (T << 32);
                t_seen = now;
            } else if (now - t_seen > 1000000000ull) {
                if (lane == 0) atomicOr((int *)&pc->state.v, 1);
                break;
            }
            __builtin_amdgcn_s_sleep(32);
        }
    } else {
        __shared__ int s_nz[WAVES_PER_BLOCK][64];
        __shared__ int s_base[WAVES_PER_BLOCK][64];
        __shared__ unsigned long long s_A[WAVES_PER_BLOCK][64];
        constexpr int GATHER_HS = LOCAL ? 256 : 128;
        __shared__ int s_hk[WAVES_PER_BLOCK][GATHER_HS];
        __shared__ uint8_t s_hv[WAVES_PER_BLOCK][GATHER_HS];
        const int n = a.nlight;
        // per-edge counts: this wave's table of member-pair edge ids
        int *etab_w = EDGE ? a.weid + (long long)(blockIdx.x * WAVES_PER_BLOCK + wv) * 4096 : nullptr;
        if (EDGE) vs.set_table(etab_w);
        for (;;) {
            const int idx = claim.next(cursor, n, claim_n0, claim_nch, lane, a.abort);
            if (idx < 0) break;
            const int v = a.order[a.light_base + idx];
            gs.set_vertex(v);
            int d, gid;
            PT_MARK(t_g);
            const uint64_t A = gather_light<GATHER_HS>(v, lane, a, s_nz[wv], s_base[wv], s_A[wv], s_hk[wv], s_hv[wv], d, gid,
                                            etab_w);
            int uni = -1;
            int2 pref = make_int2(0, 0);
            if (d > a.dfs_max) {
                uni = make_universe<KL, LK>(A, d, gid, lane, a, v, -1, 0ull, 0ull, nullptr, 0, pref, etab_w);
                if (uni < 0) continue;  // buffers full: the host reruns with larger ones
            }
            PT_ADD(7, t_g);
            PT_MARK(t_c);
            const int root = (uni < 0) ? v : -1;
            // light roots walk small trees (about 13 nodes on average on a
            // power-law graph) and rarely fill a lane batch: the lane tier is
            // compiled out of this kernel, which keeps its registers and LDS
            // for occupancy (1M-vertex graph: 6.2 -> 4.8 ms global, 11.1 ->
            // 6.1 ms per vertex)
            compact_run<KL, LK, false>(A, (d == 64) ? ~0ull : ((1ull << d) - 1), 0ull, 0ull, 1, 0, uni, d, gid,
                            root, pref, lane, a, gs, vs, ct);
            PT_ADD(8, t_c);
            PT_MARK(t_f);
            if (LOCAL) vs.flush(lane, d, gid, root, pref, uni, a);
            PT_ADD(9, t_f);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < LDS_H * 64; i += blockDim.x) {
        const int h = i >> 6, p = i & 63;
        if (s_bins[i] && h < a.hd && p < a.hd) atomicAdd(&a.hist[(long long)h * a.hd + p], s_bins[i]);
    }
    if (lane == 0) {
        atomicAdd(&a.counters[0], ct.nodes);
        atomicAdd(&a.counters[1], gs.leaves);
        atomicAdd(&a.counters[2], ct.work);
        if constexpr (MODE == PV_UNITS_ALL) {
            for (int k = 0; k < 3; k++)
                if (wk[k]) atomicAdd(&a.counters[4 + k], wk[k]);
        } else {
            atomicAdd(&a.counters[4 + MODE], ct.work);
        }
        if (ct.child) atomicAdd(&a.counters[PV_CTR_CHILD], ct.child);
#ifdef PV_PHASE_TIMING
        if (a.phase) {
            PT_ADD(12, pt_kernel0);
            pt[15] = 1;  // waves
            pt[11] = pt_sub()[0];
            if (MODE != 0) pt[10] = pt_sub()[1];  // (kind 0 keeps slot 10 for its re-index)
            pt[13] = pt_sub()[2];  // lane-batch loop trips and the nodes their lanes visited
            pt[14] = pt_sub()[3];
            for (int i = 0; i < PT_N; i++)
                if (pt[i]) atomicAdd(&a.phase[(MODE < 3 ? MODE : 0) * PT_N + i], (unsigned long long)pt[i]);
        }
#endif
    }
}

// Per-edge counts: pairs with a vertex above a universe, once per universe
// after the last level (a wave per universe).  Members add their sums
// toward hold / pivot prefix vertices; every prefix pair gets the
// universe's HH, HP or PP total by the roles of its two ends.
__global__ void __launch_bounds__(256) edge_prefix_kernel(const LevelArgs *__restrict__ pa) {
    const LevelArgs &a = *pa;
    const int lane = threadIdx.x & 63;
    const int nu = min(*a.u_n, a.u_cap);
    const int K = a.K;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    bool ovf = false;
    for (int u = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; u < nu; u += nwaves) {
        const int gid = a.u_gid[(long long)u * 64 + lane];
        const int2 pref = a.u_pref[u];
        for (int i = 0; i < pref.y; i++) {
            const int ex = a.pref_pool[pref.x + i];
            const int x = ex & 0x7fffffff, role = (ex >> 31) & 1;
            if (gid < 0) continue;
            const uint64_t *src = a.umem + 2 * ((((long long)u * 64 + lane) * 2 + role) * K);
            int e = -2;
            for (int kk = 0; kk < K; kk += a.epk ? 2 : 1) {
                const uint64_t l = src[2 * kk], hv = src[2 * kk + 1];
                const uint64_t l1 = (a.epk && kk + 1 < K) ? src[2 * kk + 2] : 0ull;
                const uint64_t h1 = (a.epk && kk + 1 < K) ? src[2 * kk + 3] : 0ull;
                if ((l | hv | l1 | h1) == 0) continue;
                if (e == -2) {
                    e = edge_id(x, gid, a.sub, a.orow, a.ocol, a.o2e);
                    if (e < 0) atomicOr(a.flags, 4);
                }
                if (e < 0) continue;
                uint64_t *dst = a.vout + 2 * ((long long)e * a.kstride + kk);
                if (a.epk) ovf |= packed_add(a.epk, a.ewrap, a.kws, e, kk / 2, l, hv, l1, h1, dst, kk + 1 < K);
                else ovf |= atomic_add_u128(dst, l, hv);
            }
        }
        const uint64_t *tot = a.utot + 2 * ((long long)u * 3 * K);
        for (int i = 0; i + 1 < pref.y; i++) {
            const int ex = a.pref_pool[pref.x + i];
            for (int j = i + 1 + lane; j < pref.y; j += 64) {
                const int ey = a.pref_pool[pref.x + j];
                const int type = ((ex >> 31) & 1) + ((ey >> 31) & 1);
                const int e = edge_id(ex & 0x7fffffff, ey & 0x7fffffff, a.sub, a.orow, a.ocol, a.o2e);
                if (e < 0) {
                    atomicOr(a.flags, 4);
                    continue;
                }
                for (int kk = 0; kk < K; kk += a.epk ? 2 : 1) {
                    const uint64_t l = tot[2 * (type * K + kk)], hv = tot[2 * (type * K + kk) + 1];
                    uint64_t *dst = a.vout + 2 * ((long long)e * a.kstride + kk);
                    if (a.epk) {
                        const bool in1 = kk + 1 < K;
                        const uint64_t l1 = in1 ? tot[2 * (type * K + kk + 1)] : 0ull;
                        const uint64_t h1 = in1 ? tot[2 * (type * K + kk + 1) + 1] : 0ull;
                        ovf |= packed_add(a.epk, a.ewrap, a.kws, e, kk / 2, l, hv, l1, h1, dst, in1);
                    } else if (l | hv) {
                        ovf |= atomic_add_u128(dst, l, hv);
                    }
                }
            }
        }
    }
    if (ovf) atomicOr(a.lovf, 1);
}

// Local counts from the packed table, added to the output once the walk
// is done.  Half 0 of a word has taken b + sum of its k = 2i charges modulo
// 2^32, each wrap counted in the low half of the word's carry count, and
// passed every such wrap on to half 1; half 1 has taken b + its k = 2i + 1
// charges plus those wraps modulo 2^32, each wrap out of the word counted in
// the high half of the carry count.  So with b the halves' starting value,
//   sum(k = 2i)     = half0 + 2^32 * wraps0 - b,
//   sum(k = 2i + 1) = half1 + 2^32 * wraps1 - wraps0 - b,
// exactly, as every count is below 2^62.
__global__ void __launch_bounds__(256) local_unpack_kernel(const uint64_t *__restrict__ epk,
                                                          const uint64_t *__restrict__ ewrap, long long words,
                                                          int kw, int kws, int K, uint64_t *__restrict__ vout,
                                                          int kstride, uint32_t bias) {
    const uint64_t start = (uint64_t)bias | ((uint64_t)bias << 32);
    for (long long w = blockIdx.x * 256ll + threadIdx.x; w < words; w += (long long)gridDim.x * 256) {
        const long long e = w / kw;
        const int i = (int)(w - e * kw);
        const uint64_t x = epk[e * kws + i], c = ewrap[e * kws + i];
        if (x == start && c == 0) continue;
        const int k0 = 2 * i;
        const uint64_t w0 = c & 0xffffffffull, w1 = c >> 32;
        const uint64_t s0 = (x & 0xffffffffull) + (w0 << 32) - bias;
        const uint64_t s1 = (x >> 32) + (w1 << 32) - w0 - bias;
        uint64_t *row = vout + 2 * (e * kstride + k0);
        uint64_t lo = row[0] + s0;
        row[1] += (lo < s0) ? 1ull : 0ull;
        row[0] = lo;
        if (k0 + 1 < K) {
            lo = row[2] + s1;
            row[3] += (lo < s1) ? 1ull : 0ull;
            row[2] = lo;
        }
    }
}

// Per-vertex counts: what each universe's walks owe the vertices above it
// (its prefix: the root, then hold or pivot vertices), added once after the
// last level.  The universes of one heavy root share most of their prefix
// (siblings differ in one vertex), so adding every entry straight to HBM
// makes their atomics on one line wait for each other.  Instead the
// universes are grouped by heavy root, each group's totals are summed per
// prefix vertex in LDS, and each sum reaches HBM with one atomic per k.
// In the pool, a multi-word universe's entries after the root are local
// indices into N+(root) (oriented CSR order); other universes hold the root
// alone.

// 128-bit add into LDS (two 64-bit atomics, the carry between them)
__device__ __forceinline__ bool lds_add_u128(uint64_t *p, uint64_t lo, uint64_t hi) {
    bool ovf = false;
    if (lo) {
        const uint64_t old = __hip_atomic_fetch_add(p, lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old + lo < old) {
            hi += 1;
            if (hi == 0) ovf = true;
        }
    }
    if (hi) {
        const uint64_t old = __hip_atomic_fetch_add(p + 1, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old + hi < old) ovf = true;
    }
    return ovf;
}

// Pass 1: each grouped universe takes its position in its heavy root's
// group (one counter atomic per distinct group of a wave); a universe of a
// light root adds its totals to the root directly.
__global__ void __launch_bounds__(256) prefix_count_kernel(const LevelArgs *__restrict__ pa,
                                                           int *__restrict__ gcnt, int *__restrict__ gpos) {
    const LevelArgs &a = *pa;
    const int lane = threadIdx.x & 63;
    const int nu = min(*a.u_n, a.u_cap);
    const int K = a.K;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    bool ovf = false;
    for (int u0 = blockIdx.x * blockDim.x; u0 < nu; u0 += gridDim.x * blockDim.x) {
        const int u = u0 + (int)threadIdx.x;
        const int g = (u < nu) ? a.u_grp[u] : -1;
        bool pending = g >= 0;
        for (uint64_t bl = ballot64(pending); bl; bl = ballot64(pending)) {
            const int lead = __builtin_ctzll(bl);
            const int lg = (int)readlane32((uint32_t)g, lead);
            const bool mine = pending && g == lg;
            const uint64_t m = ballot64(mine);
            int base = 0;
            if (lane == lead) base = atomicAdd(&gcnt[lg], __popcll(m));
            base = (int)readlane32((uint32_t)base, lead);
            if (mine) {
                gpos[u] = base + __popcll(m & below);
                pending = false;
            }
        }
        if (u < nu && g < 0) {
            const int2 pref = a.u_pref[u];
            const uint64_t *tot = a.utot + 2 * ((long long)u * 2 * K);
            for (int i = 0; i < pref.y; i++) {
                const int e = a.pref_pool[pref.x + i];
                const uint64_t *t = tot + (((e >> 31) & 1) ? 2 * K : 0);
                uint64_t *dst = a.vout + 2 * ((long long)(e & 0x7fffffff) * a.kstride);
                uint64_t lo[PV_MAX_LOCAL_K], old[PV_MAX_LOCAL_K];
#pragma unroll
                for (int kk = 0; kk < PV_MAX_LOCAL_K; kk++) {
                    lo[kk] = (kk < K) ? t[2 * kk] : 0ull;
                    old[kk] = atomic_add_u128_lo(dst + 2 * kk, lo[kk]);
                }
#pragma unroll
                for (int kk = 0; kk < PV_MAX_LOCAL_K; kk++) asm volatile("" : "+v"(old[kk]));
#pragma unroll
                for (int kk = 0; kk < PV_MAX_LOCAL_K; kk++)
                    if (kk < K) ovf |= atomic_add_u128_hi(dst + 2 * kk, lo[kk], old[kk], t[2 * kk + 1]);
            }
        }
    }
    if (ovf) atomicOr(a.lovf, 1);
}

// Pass 3: universes listed group by group
__global__ void __launch_bounds__(256) prefix_scatter_kernel(const LevelArgs *__restrict__ pa,
                                                             const int *__restrict__ goff,
                                                             const int *__restrict__ gpos,
                                                             int *__restrict__ glist) {
    const LevelArgs &a = *pa;
    const int nu = min(*a.u_n, a.u_cap);
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < nu; u += gridDim.x * blockDim.x) {
        const int g = a.u_grp[u];
        if (g >= 0) glist[goff[g] + gpos[u]] = u;
    }
}

// Pass 4: a workgroup takes PV_PREFIX_SLICE consecutive entries of the
// grouped list; per group segment it sums the totals owed to each prefix
// vertex in LDS (rows: N+(root) indices r0 .. r0+rows-1 per pass, plus one
// row for the root) and adds the nonzero sums to HBM.
__global__ void __launch_bounds__(256) prefix_group_kernel(const LevelArgs *__restrict__ pa, int ngroups,
                                                           const int *__restrict__ goff,
                                                           const int *__restrict__ glist, int rows) {
    __shared__ uint64_t s_acc[2 * PV_PREFIX_SLOTS];
    const LevelArgs &a = *pa;
    const int K = a.K, ks = a.kstride;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
    // a wave adds E = 64 / K prefix entries side by side: lane = slot * K + kk
    const int E = 64 / K;
    const int slot = lane / K, kk = lane - slot * K;
    const bool act = slot < E;
    const int R = rows;  // (R + 1) * K <= PV_PREFIX_SLOTS
    const int total = goff[ngroups];
    bool ovf = false;
    for (int p0 = blockIdx.x * PV_PREFIX_SLICE; p0 < total; p0 += gridDim.x * PV_PREFIX_SLICE) {
        const int p1 = min(p0 + PV_PREFIX_SLICE, total);
        // the group holding entry p0: the last g with goff[g] <= p0
        int lo = 0, hi = ngroups - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (goff[mid] <= p0) lo = mid; else hi = mid - 1;
        }
        for (int g = lo; g < ngroups && goff[g] < p1; g++) {
            const int q0 = max(p0, goff[g]), q1 = min(p1, goff[g + 1]);
            if (q0 >= q1) continue;
            const int root = a.order[g];
            const int rb = a.orow[root], d = a.orow[root + 1] - rb;
            for (int r0 = 0; r0 == 0 || r0 < d; r0 += R) {
                // rows in use: local indices r0 .. r0+nr-1, then the root's row
                const int nr = max(0, min(R, d - r0));
                const int nslot = (nr + 1) * K;
                for (int i = threadIdx.x; i < nslot; i += blockDim.x) {
                    const bool mem = i < nr * K;
                    const int row = mem ? i / K : R;
                    const int j = row * K + (mem ? i - row * K : i - nr * K);
                    s_acc[2 * j] = 0ull;
                    s_acc[2 * j + 1] = 0ull;
                }
                __syncthreads();
                for (int q = q0 + wv; q < q1; q += nwv) {
                    const int u = glist[q];
                    const int2 pref = a.u_pref[u];
                    if (!act) continue;
                    const uint64_t *tot = a.utot + 2 * ((long long)u * 2 * K);
                    const uint64_t hl = tot[2 * kk], hh = tot[2 * kk + 1];
                    const uint64_t pl = tot[2 * (K + kk)], ph = tot[2 * (K + kk) + 1];
                    if ((hl | hh | pl | ph) == 0) continue;
                    for (int i = slot; i < pref.y; i += E) {
                        const int e = a.pref_pool[pref.x + i];
                        int row = -1;
                        if (i == 0) {
                            if (r0 == 0) row = R;  // the root (a global id)
                        } else {
                            const int jj = (e & 0x7fffffff) - r0;
                            if (jj >= 0 && jj < nr) row = jj;
                        }
                        if (row < 0) continue;
                        const bool isP = (e >> 31) & 1;
                        ovf |= lds_add_u128(&s_acc[2 * (row * K + kk)], isP ? pl : hl, isP ? ph : hh);
                    }
                }
                __syncthreads();
                for (int i = threadIdx.x; i < nslot; i += blockDim.x) {
                    const bool mem = i < nr * K;
                    const int row = mem ? i / K : R;
                    const int k2 = mem ? i - row * K : i - nr * K;
                    const uint64_t l = s_acc[2 * (row * K + k2)], h = s_acc[2 * (row * K + k2) + 1];
                    if ((l | h) == 0) continue;
                    const int x = mem ? a.ocol[rb + r0 + row] : root;
                    ovf |= atomic_add_u128(a.vout + 2 * ((long long)x * ks + k2), l, h);
                }
                __syncthreads();
            }
        }
    }
    if (ovf) atomicOr(a.lovf, 1);
}

// Roots with an empty out-neighbourhood are leaves (h=1, p=0) of the SCT.
__global__ void sct_sink_roots_kernel(int n, const int *__restrict__ order, const int *__restrict__ bounds,
                                      unsigned long long *hist, int hd, unsigned long long *counters,
                                      uint64_t *vout, int klo, int kstride, const int *__restrict__ vgraph) {
    const int first = bounds[1];
    const int cnt = n - first;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && cnt > 0) {
        if (!vgraph) atomicAdd(&hist[1 * hd + 0], (unsigned long long)cnt);
        atomicAdd(&counters[0], (unsigned long long)cnt);
        atomicAdd(&counters[1], (unsigned long long)cnt);
    }
    if (vgraph) {
        // batch: each sink root is a leaf of its own graph's tree
        for (int j = i; j < cnt; j += gridDim.x * blockDim.x) {
            const int v = order[first + j];
            atomicAdd(&hist[(long long)vgraph[v] * hd * hd + 1 * hd + 0], 1ull);
        }
    }
    if (vout && klo == 1) {
        for (int j = i; j < cnt; j += gridDim.x * blockDim.x) {
            const int v = order[first + j];
            atomicAdd((unsigned long long *)(vout + 2 * ((long long)v * kstride)), 1ull);
        }
    }
}

// Leaf moments of the (h, p) histograms: each thread a strided share of the
// cells, then a block reduction and one atomic per block and sum.
__global__ void __launch_bounds__(256) leaf_moments_kernel(const unsigned long long *__restrict__ hist,
                                                           long long cells, int hd,
                                                           unsigned long long *counters) {
    __shared__ unsigned long long s_hp[256], s_pp[256];
    unsigned long long hp = 0, pp = 0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < cells;
         i += (long long)gridDim.x * blockDim.x) {
        const unsigned long long L = hist[i];
        if (!L) continue;
        const int c = (int)(i % ((long long)hd * hd));
        const int h = c / hd, p = c % hd;
        hp += L * (unsigned long long)(h + p);
        pp += L * (unsigned long long)(p + 1);
    }
    s_hp[threadIdx.x] = hp;
    s_pp[threadIdx.x] = pp;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_hp[threadIdx.x] += s_hp[threadIdx.x + w];
            s_pp[threadIdx.x] += s_pp[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (s_hp[0]) atomicAdd(&counters[PV_CTR_HP], s_hp[0]);
        if (s_pp[0]) atomicAdd(&counters[PV_CTR_PP], s_pp[0]);
    }
}

// ============================================================== finalize
// Exact binomials (Pascal's rule) in u128 with a flag for values >= 2^128,
// and a u64 copy of the first 16 columns for the per-vertex path.

__global__ void binom_kernel(int bn, uint64_t *tab, uint8_t *bad, uint64_t *tab64, int *fits64) {
    // one block: row by row
    for (int a = 0; a < bn; a++) {
        for (int b = threadIdx.x; b < bn; b += blockDim.x) {
            uint64_t lo = 0, hi = 0;
            uint8_t bd = 0;
            if (b == 0) lo = 1;
            else if (b <= a) {
                const long long i1 = (long long)(a - 1) * bn + (b - 1);
                const long long i2 = (long long)(a - 1) * bn + b;
                uint64_t xl = tab[2 * i1], xh = tab[2 * i1 + 1];
                uint64_t yl = (b <= a - 1) ? tab[2 * i2] : 0, yh = (b <= a - 1) ? tab[2 * i2 + 1] : 0;
                bd = bad[i1] | ((b <= a - 1) ? bad[i2] : 0);
                lo = xl + yl;
                const uint64_t c = (lo < xl) ? 1 : 0;
                hi = xh + yh;
                if (hi < xh) bd = 1;
                const uint64_t hi2 = hi + c;
                if (hi2 < hi) bd = 1;
                hi = hi2;
            }
            tab[2 * ((long long)a * bn + b)] = lo;
            tab[2 * ((long long)a * bn + b) + 1] = hi;
            bad[(long long)a * bn + b] = bd;
            if (b < 16) {
                tab64[(long long)a * 16 + b] = lo;
                if (hi != 0 || bd) atomicAnd(&fits64[b], 0);
            }
        }
        __syncthreads();
    }
}

// Padded 64-bit table for the per-vertex path (see VertexSink): row a =
// -1..bn-1, column j = -16..ts-17 at [(a + 1) * ts + j + 16].
__global__ void binom_pad_kernel(int bn, int ts, const uint64_t *__restrict__ tab, const uint8_t *__restrict__ bad,
                                 uint64_t *__restrict__ pad) {
    // low limbs at pad[0, total), high limbs at pad[total, 2 total); an
    // entry that reaches 2^128 holds all ones in both (the sinks flag it)
    const int total = (bn + 1) * ts;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int a = i / ts - 1, j = i % ts - 16;
        const bool in = a >= 0 && j >= 0 && j <= a;
        const long long t = (long long)a * bn + j;
        const bool b = in && bad[t];
        pad[i] = b ? ~0ull : (in ? tab[2 * t] : 0ull);
        pad[total + i] = b ? ~0ull : (in ? tab[2 * t + 1] : 0ull);
    }
}

// C_k = sum_{h,p} L[h][p] * C(p, k-h), exact u128 with overflow detection;
// one block per k.
__global__ void __launch_bounds__(256) finalize_kernel(const unsigned long long *__restrict__ hist,
                                                        int hd, const uint64_t *__restrict__ tab,
                                                        const uint8_t *__restrict__ bad, int bn,
                                                        int kmax, int c0, uint64_t *counts,
                                                        uint64_t *ovf_words, int *omega) {
    __shared__ uint64_t s_lo[256], s_hi[256];
    __shared__ int s_ovf[256];
    const int k = blockIdx.x;
    // batch: graph blockIdx.y has its own histogram, counts row and flags
    const int gb = blockIdx.y;
    hist += (long long)gb * hd * hd;
    counts += (long long)gb * gridDim.x * 2;
    ovf_words += (long long)gb * ((gridDim.x + 63) / 64);
    omega += gb;
    uint64_t lo = 0, hi = 0;
    int ovf = 0;
    for (int p = threadIdx.x; p < hd; p += blockDim.x) {
        const int h0 = max(1, k - p);
        for (int h = h0; h <= k && h < hd; h++) {
            const unsigned long long L = hist[(long long)h * hd + p];
            if (!L) continue;
            const int i = k - h;  // 0 <= i <= p
            if (p >= bn) { ovf = 1; continue; }
            const long long ti = (long long)p * bn + i;
            if (bad[ti]) ovf = 1;
            const uint64_t bl = tab[2 * ti], bh = tab[2 * ti + 1];
            // (L * (bh:bl)) must fit 128 bits
            const uint64_t p0l = (uint64_t)L * bl;
            const uint64_t p0h = __umul64hi((uint64_t)L, bl);
            const uint64_t p1l = (uint64_t)L * bh;
            const uint64_t p1h = __umul64hi((uint64_t)L, bh);
            if (p1h) ovf = 1;
            const uint64_t th = p0h + p1l;
            if (th < p0h) ovf = 1;
            const uint64_t nlo = lo + p0l;
            const uint64_t carry = (nlo < lo) ? 1 : 0;
            uint64_t nhi = hi + th;
            if (nhi < hi) ovf = 1;
            const uint64_t nhi2 = nhi + carry;
            if (nhi2 < nhi) ovf = 1;
            lo = nlo;
            hi = nhi2;
        }
    }
    s_lo[threadIdx.x] = lo;
    s_hi[threadIdx.x] = hi;
    s_ovf[threadIdx.x] = ovf;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t a = 0, b = 0;
        int o = 0;
        for (int t = 0; t < (int)blockDim.x; t++) {
            const uint64_t nl = a + s_lo[t];
            const uint64_t c = (nl < a) ? 1 : 0;
            const uint64_t nh = b + s_hi[t];
            if (nh < b) o = 1;
            const uint64_t nh2 = nh + c;
            if (nh2 < nh) o = 1;
            a = nl;
            b = nh2;
            o |= s_ovf[t];
        }
        if (k == 0) { a = (uint64_t)c0; b = 0; o = 0; }
        if (kmax > 0 && k > kmax) { a = 0; b = 0; o = 0; }
        counts[2 * k] = a;
        counts[2 * k + 1] = b;
        if (o) atomicOr((unsigned long long *)&ovf_words[k >> 6], 1ull << (k & 63));
        if (k > 0 && ((a | b) || o)) atomicMax(omega, k);
    }
}

// ------------------------------------------------ counts wider than u128
// The same read-off (Sec. 5: C_k = sum over leaves (h, p) of C(p, k - h))
// in little-endian 64-bit limbs, for graphs whose counts pass 2^128.

// largest h + p over the nonzero histogram bins (a leaf's H and P form a
// clique, so every binomial needed has p <= that bound)
__global__ void __launch_bounds__(256) hist_span_kernel(const unsigned long long *__restrict__ hist, int hd,
                                                        int *out) {
    int best = 0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < (long long)hd * hd;
         i += (long long)gridDim.x * blockDim.x) {
        const int h = (int)(i / hd), p = (int)(i % hd);
        if (hist[i]) best = max(best, h + p);
    }
    best = wave_max_i32(best);
    if ((threadIdx.x & 63) == 0 && best > 0) atomicMax(out, best);
}

// C(p, j) for 0 <= j <= p < bn in `limbs` limbs (C(p, j) < 2^p <= 2^(64
// limbs)), row by row by Pascal's rule; one workgroup
__global__ void __launch_bounds__(256) binom_wide_kernel(int bn, int limbs, uint64_t *tab) {
    for (int p = 0; p < bn; p++) {
        for (int j = threadIdx.x; j < bn; j += blockDim.x) {
            uint64_t *d = tab + ((long long)p * bn + j) * limbs;
            if (j > p) {
                for (int l = 0; l < limbs; l++) d[l] = 0ull;
            } else if (j == 0 || j == p) {
                d[0] = 1ull;
                for (int l = 1; l < limbs; l++) d[l] = 0ull;
            } else {
                const uint64_t *a = tab + ((long long)(p - 1) * bn + j - 1) * limbs;
                const uint64_t *b = a + limbs;  // C(p-1, j)
                uint64_t c = 0;
                for (int l = 0; l < limbs; l++) {
                    const uint64_t x = a[l] + b[l];
                    const uint64_t y = x + c;
                    c = (x < a[l] ? 1ull : 0ull) + (y < x ? 1ull : 0ull);
                    d[l] = y;
                }
            }
        }
        __syncthreads();
    }
}

// One workgroup per k: thread t < W owns limb t as a 128-bit carry-save
// sum (the low half of L * B[t] and the high half of L * B[t-1] over all
// leaf bins); thread 0 then propagates the carries.  W = table limbs + 1
// holds any count (the histogram total is below 2^64).  out: [kcap][W].
__global__ void __launch_bounds__(128) finalize_wide_kernel(const unsigned long long *__restrict__ hist, int hd,
                                                            const uint64_t *__restrict__ tab, int bn, int tl,
                                                            int W, int kmax, int c0, uint64_t *out, int *omega) {
    __shared__ uint64_t s_lo[128], s_hi[128];
    const int k = blockIdx.x;
    const int t = threadIdx.x;
    uint64_t lo = 0, hi = 0;
    if (t < W && k > 0 && (kmax <= 0 || k <= kmax)) {
        for (int h = 1; h <= k && h < hd; h++) {
            const int j = k - h;  // C(p, j) with p >= j
            for (int p = j; p < bn && p < hd; p++) {
                const unsigned long long L = hist[(long long)h * hd + p];
                if (!L) continue;
                const uint64_t *B = tab + ((long long)p * bn + j) * tl;
                const uint64_t b0 = (t < tl) ? B[t] : 0ull;
                const uint64_t b1 = (t >= 1 && t - 1 < tl) ? B[t - 1] : 0ull;
                const uint64_t a = (uint64_t)L * b0;            // low half of L * B[t]
                const uint64_t c = __umul64hi((uint64_t)L, b1);  // high half of L * B[t-1]
                const uint64_t n1 = lo + a;
                hi += (n1 < lo) ? 1ull : 0ull;
                const uint64_t n2 = n1 + c;
                hi += (n2 < n1) ? 1ull : 0ull;
                lo = n2;
            }
        }
    }
    if (t < 128) {
        s_lo[t] = lo;
        s_hi[t] = hi;
    }
    __syncthreads();
    if (t == 0) {
        uint64_t cl = 0, ch = 0;  // carry into the current limb (128-bit)
        bool any = false;
        for (int l = 0; l < W; l++) {
            const uint64_t x = s_lo[l] + cl;
            const uint64_t c1 = (x < cl) ? 1ull : 0ull;
            out[(long long)k * W + l] = x;
            any = any || x;
            // next carry = s_hi[l] + ch + c1 (fits: far below 2^128)
            const uint64_t y = s_hi[l] + ch;
            cl = y + c1;
            ch = (y < s_hi[l] ? 1ull : 0ull) + (cl < y ? 1ull : 0ull);
        }
        if (k == 0) {
            out[0] = (uint64_t)c0;
            for (int l = 1; l < W; l++) out[l] = 0ull;
        } else if (any) {
            atomicMax(omega, k);
        }
    }
}

hipError_t pv_launch_count_wide(const unsigned long long *hist, int hd, int kcap, int kmax, int c0, int *span,
                                uint64_t *tab, int bn, int tl, int W, uint64_t *out, int *omega, int phase,
                                hipStream_t s) {
    if (phase == 0) {
        hist_span_kernel<<<std::max(1, std::min(1024, (hd * hd + 255) / 256)), 256, 0, s>>>(hist, hd, span);
        return hipGetLastError();
    }
    binom_wide_kernel<<<1, 256, 0, s>>>(bn, tl, tab);
    finalize_wide_kernel<<<kcap, 128, 0, s>>>(hist, hd, tab, bn, tl, W, kmax, c0, out, omega);
    return hipGetLastError();
}

// ============================================================== host side

template <int KL, int LK>
static hipError_t launch_mode(const LevelArgs *a, int mode, int blocks, hipStream_t s) {
    dim3 g(blocks), b(64 * WAVES_PER_BLOCK);
    if (mode == PV_UNITS_MW) sct_level_kernel<KL, PV_UNITS_MW, LK><<<g, b, 0, s>>>(a);
    else if (mode == PV_UNITS_ITEMS) sct_level_kernel<KL, PV_UNITS_ITEMS, LK><<<g, b, 0, s>>>(a);
    else if (mode == PV_UNITS_LIGHT) sct_level_kernel<KL, PV_UNITS_LIGHT, LK><<<g, b, 0, s>>>(a);
    else sct_level_kernel<KL, PV_UNITS_ALL, LK><<<g, b, 0, s>>>(a);
    return hipGetLastError();
}

// kl: 0 (global counts only), 8 or 16 k-slots; lk: PV_LK_*
hipError_t pv_launch_level(const LevelArgs *a, int kl, int lk, int mode, int blocks, hipStream_t s) {
    if (kl == 0) return launch_mode<0, PV_LK_VERTEX128>(a, mode, blocks, s);
    if (lk == PV_LK_EDGE) return launch_mode<8, PV_LK_EDGE>(a, mode, blocks, s);
    if (kl <= 8)
        return lk == PV_LK_VERTEX64 ? launch_mode<8, PV_LK_VERTEX64>(a, mode, blocks, s)
                                    : launch_mode<8, PV_LK_VERTEX128>(a, mode, blocks, s);
    return lk == PV_LK_VERTEX64 ? launch_mode<16, PV_LK_VERTEX64>(a, mode, blocks, s)
                                : launch_mode<16, PV_LK_VERTEX128>(a, mode, blocks, s);
}

template <int KL, int LK>
static int blocks_per_cu_kl(int mode) {
    int nb = 0;
    hipError_t e;
    if (mode == PV_UNITS_MW)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sct_level_kernel<KL, PV_UNITS_MW, LK>,
                                                         64 * WAVES_PER_BLOCK, 0);
    else if (mode == PV_UNITS_ITEMS)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sct_level_kernel<KL, PV_UNITS_ITEMS, LK>,
                                                         64 * WAVES_PER_BLOCK, 0);
    else if (mode == PV_UNITS_LIGHT)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sct_level_kernel<KL, PV_UNITS_LIGHT, LK>,
                                                         64 * WAVES_PER_BLOCK, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sct_level_kernel<KL, PV_UNITS_ALL, LK>,
                                                         64 * WAVES_PER_BLOCK, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

int pv_level_blocks_per_cu(int kl, int lk, int mode) {
    if (kl == 0) return blocks_per_cu_kl<0, PV_LK_VERTEX128>(mode);
    if (lk == PV_LK_EDGE) return blocks_per_cu_kl<8, PV_LK_EDGE>(mode);
    if (kl <= 8)
        return lk == PV_LK_VERTEX64 ? blocks_per_cu_kl<8, PV_LK_VERTEX64>(mode)
                                    : blocks_per_cu_kl<8, PV_LK_VERTEX128>(mode);
    return lk == PV_LK_VERTEX64 ? blocks_per_cu_kl<16, PV_LK_VERTEX64>(mode)
                                : blocks_per_cu_kl<16, PV_LK_VERTEX128>(mode);
}

hipError_t pv_launch_edge_prefix(const LevelArgs *a, int blocks, hipStream_t s) {
    edge_prefix_kernel<<<blocks, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t pv_launch_local_unpack(const uint64_t *epk, const uint64_t *ewrap, long long m, int kw, int kws, int K,
                                 uint64_t *vout, int kstride, uint32_t bias, int num_cu, hipStream_t s) {
    const long long words = m * kw;
    if (words <= 0) return hipSuccess;
    const int blocks = (int)std::min<long long>((words + 255) / 256, (long long)num_cu * 8);
    local_unpack_kernel<<<blocks, 256, 0, s>>>(epk, ewrap, words, kw, kws, K, vout, kstride, bias);
    return hipGetLastError();
}

hipError_t pv_launch_vertex_prefix(const LevelArgs *a, int max_units, int ngroups, const PrefixWork &w,
                                   int rows, hipStream_t s) {
    if (max_units <= 0) return hipSuccess;
    const int ub = (max_units + 255) / 256;
    hipError_t e = hipSuccess;
    if (ngroups > 0 && (e = hipMemsetAsync(w.gcnt, 0, (size_t)ngroups * sizeof(int), s)) != hipSuccess) return e;
    prefix_count_kernel<<<ub, 256, 0, s>>>(a, w.gcnt, w.gpos);
    if (ngroups <= 0) return hipGetLastError();
    if ((e = pv_launch_excl_scan(ngroups, w.gcnt, w.scan_tmp, w.goff, s)) != hipSuccess) return e;
    prefix_scatter_kernel<<<ub, 256, 0, s>>>(a, w.goff, w.gpos, w.glist);
    prefix_group_kernel<<<(max_units + PV_PREFIX_SLICE - 1) / PV_PREFIX_SLICE, 256, 0, s>>>(a, ngroups, w.goff,
                                                                                           w.glist, rows);
    return hipGetLastError();
}

hipError_t pv_launch_sink_roots(int n, const int *order, const int *bounds, unsigned long long *hist,
                                int hd, unsigned long long *counters, uint64_t *vout, int klo, int kstride,
                                const int *vgraph, hipStream_t s) {
    sct_sink_roots_kernel<<<256, 256, 0, s>>>(n, order, bounds, hist, hd, counters, vout, klo, kstride, vgraph);
    return hipGetLastError();
}

hipError_t pv_launch_binomials(int bn, uint64_t *tab128, uint8_t *bad, uint64_t *tab64, int *fits64,
                               hipStream_t s) {
    binom_kernel<<<1, 256, 0, s>>>(bn, tab128, bad, tab64, fits64);
    return hipGetLastError();
}

hipError_t pv_launch_binom_pad(int bn, int ts, const uint64_t *tab128, const uint8_t *bad, uint64_t *pad,
                               hipStream_t s) {
    binom_pad_kernel<<<64, 256, 0, s>>>(bn, ts, tab128, bad, pad);
    return hipGetLastError();
}

hipError_t pv_launch_finalize(const unsigned long long *hist, int hd, const uint64_t *tab128,
                              const uint8_t *bad, int bn, int kcap, int kmax, int c0,
                              uint64_t *counts, uint64_t *ovf_words, int *omega, int graphs,
                              hipStream_t s) {
    finalize_kernel<<<dim3(kcap, graphs), 256, 0, s>>>(hist, hd, tab128, bad, bn, kmax, c0, counts,
                                                      ovf_words, omega);
    return hipGetLastError();
}

hipError_t pv_launch_leaf_moments(const unsigned long long *hist, int hd, int graphs,
                                  unsigned long long *counters, hipStream_t s) {
    const long long cells = (long long)graphs * hd * hd;
    const long long b = (cells + 4095) / 4096;
    leaf_moments_kernel<<<(int)(b < 1 ? 1 : (b > 1024 ? 1024 : b)), 256, 0, s>>>(hist, cells, hd, counters);
    return hipGetLastError();
}
