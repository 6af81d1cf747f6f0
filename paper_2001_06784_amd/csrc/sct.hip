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

// ------------------------------------------------------------------ sinks

// Global counts: leaf (h,p) -> L[h][p] += 1.  Lane l keeps L[h][l] for
// h = 1..8 in registers; other leaves go straight to the device histogram.
struct GlobalSink {
    uint32_t c1, c2, c3, c4, c5, c6, c7, c8;
    uint32_t pending;  // leaves since the last flush (wave-uniform)
    unsigned long long leaves;

    __device__ void reset() {
        c1 = c2 = c3 = c4 = c5 = c6 = c7 = c8 = 0;
        pending = 0;
    }

    __device__ void flush(int lane, unsigned long long *hist, int hd) {
        if (lane < hd) {
            if (c1) atomicAdd(&hist[1 * hd + lane], (unsigned long long)c1);
            if (c2 && 2 < hd) atomicAdd(&hist[2 * hd + lane], (unsigned long long)c2);
            if (c3 && 3 < hd) atomicAdd(&hist[3 * hd + lane], (unsigned long long)c3);
            if (c4 && 4 < hd) atomicAdd(&hist[4 * hd + lane], (unsigned long long)c4);
            if (c5 && 5 < hd) atomicAdd(&hist[5 * hd + lane], (unsigned long long)c5);
            if (c6 && 6 < hd) atomicAdd(&hist[6 * hd + lane], (unsigned long long)c6);
            if (c7 && 7 < hd) atomicAdd(&hist[7 * hd + lane], (unsigned long long)c7);
            if (c8 && 8 < hd) atomicAdd(&hist[8 * hd + lane], (unsigned long long)c8);
        }
        reset();
    }

    __device__ __forceinline__ void leaf(int h, int p, int lane, unsigned long long *hist, int hd) {
        leaves++;
        if (h <= PV_HREG && p < 64) {
            const uint32_t inc = (lane == p) ? 1u : 0u;
            switch (h) {
                case 1: c1 += inc; break;
                case 2: c2 += inc; break;
                case 3: c3 += inc; break;
                case 4: c4 += inc; break;
                case 5: c5 += inc; break;
                case 6: c6 += inc; break;
                case 7: c7 += inc; break;
                default: c8 += inc; break;
            }
            if (++pending == 0x7fffffffu) flush(lane, hist, hd);
        } else if (lane == 0) {
            atomicAdd(&hist[(long long)h * hd + p], 1ull);
        }
    }
};

__device__ __forceinline__ uint64_t bin_at(const uint64_t *bin64, int a, int b) {
    return (b < 0 || a < 0 || b > a) ? 0ull : bin64[a * 16 + b];
}

// Per-vertex counts (Alg. 2 steps ht and pt).  Lane j accumulates the
// contributions of universe member j for k = klo..klo+K-1; lane kk < K
// accumulates the totals owed to every vertex above the universe (TH for
// hold vertices, TP for pivot vertices).
template <int KL>
struct VertexSink {
    uint64_t lo[KL > 0 ? KL : 1], hi[KL > 0 ? KL : 1];
    uint64_t thl, thh, tpl, tph;

    __device__ void reset() {
#pragma unroll
        for (int i = 0; i < KL; i++) lo[i] = hi[i] = 0;
        thl = thh = tpl = tph = 0;
    }

    __device__ __forceinline__ void leaf(int h, int p, uint64_t H, uint64_t P, int lane,
                                         const LevelArgs &a) {
        const bool inH = (H >> lane) & 1, inP = (P >> lane) & 1;
        const int kfrom = max(a.klo, h), kto = min(a.klo + a.K - 1, h + p);
#pragma unroll
        for (int kk = 0; kk < KL; kk++) {
            const int k = a.klo + kk;
            if (k >= kfrom && k <= kto) {
                const uint64_t bH = bin_at(a.bin64, p, k - h);
                const uint64_t bP = bin_at(a.bin64, p - 1, k - h - 1);
                const uint64_t v = inH ? bH : (inP ? bP : 0ull);
                lo[kk] += v;
                hi[kk] += (lo[kk] < v) ? 1ull : 0ull;
            }
        }
        if (lane < a.K) {
            const int i = a.klo + lane - h;
            const uint64_t bH = bin_at(a.bin64, p, i);
            const uint64_t bP = bin_at(a.bin64, p - 1, i - 1);
            thl += bH;
            thh += (thl < bH) ? 1ull : 0ull;
            tpl += bP;
            tph += (tpl < bP) ? 1ull : 0ull;
        }
    }

    // members: lane j < nm owns vertex gid; prefix: `root` (a hold vertex,
    // or -1) plus pool[pref.x .. pref.x + pref.y)
    __device__ void flush(int lane, int nm, int gid, int root, int2 pref, const LevelArgs &a) {
        bool ovf = false;
        if (lane < nm) {
#pragma unroll
            for (int kk = 0; kk < KL; kk++)
                if (kk < a.K && (lo[kk] | hi[kk]))
                    ovf |= atomic_add_u128(a.vout + 2 * ((long long)gid * a.K + kk), lo[kk], hi[kk]);
        }
        if (root >= 0 && lane < a.K && (thl | thh))
            ovf |= atomic_add_u128(a.vout + 2 * ((long long)root * a.K + lane), thl, thh);
        for (int i = 0; i < pref.y; i++) {
            const int e = a.pref_pool[pref.x + i];
            const int x = e & 0x7fffffff;
            const bool isP = (e >> 31) & 1;
            const uint64_t l = isP ? tpl : thl, hh = isP ? tph : thh;
            if (lane < a.K && (l | hh))
                ovf |= atomic_add_u128(a.vout + 2 * ((long long)x * a.K + lane), l, hh);
        }
        if (ovf) atomicOr(a.lovf, 1);
        reset();
    }
};

// Work counters of a wave: SCT nodes visited, and the algorithmic pivot
// work sum over nodes of |S| * ceil(|S|/64) (64-bit AND+popcount pairs).
struct Ctr {
    unsigned long long nodes, work;
};

// ------------------------------------------------------ compact-tier DFS
// Walk the whole subtree of node (S, H, P, h, p) of a compact universe
// whose row for member `lane` is A.  Depth first, stack in lane-indexed
// registers (frame t in lane t; at most 63 frames since every frame's set
// is a strict superset of the next one's).

template <int KL>
__device__ void compact_dfs(uint64_t A, uint64_t S, uint64_t H, uint64_t P, int h, int p, int lane,
                            const LevelArgs &a, GlobalSink &gs, VertexSink<KL> &vs,
                            Ctr &ct) {
    constexpr bool LOCAL = KL > 0;
    uint64_t stS = 0, stH = 0, stP = 0;
    uint32_t stM = 0;
    int depth = 0;
    for (;;) {
        ct.nodes++;
        if (S != 0) {
            const int s = __popcll(S);
            ct.work += (unsigned long long)s;
            const bool in = (S >> lane) & 1;
            const uint32_t c = (uint32_t)__popcll(A & S);
            const uint32_t key = in ? (((c + 1u) << 6) | (uint32_t)(63 - lane)) : 0u;
            const uint32_t best = wave_max_u32(key);
            const int piv = 63 - (int)(best & 63u);
            const int pc = (int)(best >> 6) - 1;
            const uint64_t pbit = 1ull << piv;
            if (pc + 1 == s) {
                // the pivot sees all of S: no hold child.  If every member
                // does, S is a clique and its pivot chain ends in one leaf.
                if (ballot64(in && (int)c + 1 != s) == 0) {
                    ct.nodes += (unsigned long long)s;
                    ct.work += (unsigned long long)s * (unsigned long long)(s - 1) / 2;
                    if (LOCAL) P |= S;
                    p += s;
                } else {
                    S &= ~pbit;
                    if (LOCAL) P |= pbit;
                    p++;
                    continue;
                }
            } else {
                const uint64_t Ap = readlane64(A, piv);
                if (!(a.kmax > 0 && h + 1 > a.kmax)) {
                    stS = writelane64(stS, S, depth);
                    if (LOCAL) {
                        stH = writelane64(stH, H, depth);
                        stP = writelane64(stP, P, depth);
                    }
                    stM = writelane32(stM, (uint32_t)piv | ((uint32_t)h << 6) | ((uint32_t)p << 19),
                                      depth);
                    depth++;
                }
                S &= Ap;
                if (LOCAL) P |= pbit;
                p++;
                continue;
            }
        }
        // a leaf: S is empty (or a clique folded into P above)
        gs.leaf(h, p, lane, a.hist, a.hd);
        if (LOCAL) vs.leaf(h, p, H, P, lane, a);
        if (depth == 0) return;
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
            H = readlane64(stH, t) | vbit;
            P = readlane64(stP, t);
        }
    }
}

// ---------------------------------------------------- compact-tier chain
// Follow the pivot chain of node (S,H,P,h,p) in universe `uni`; hold
// children go to the next level; once |S| <= dfs_max finish depth first.
// root/pref name the vertices above the universe (local counts only).

template <int KL>
__device__ void compact_run(uint64_t A, uint64_t S, uint64_t H, uint64_t P, int h, int p, int uni,
                            int nm, int gid, int root, int2 pref, int lane, const LevelArgs &a,
                            GlobalSink &gs, VertexSink<KL> &vs, Ctr &ct) {
    constexpr bool LOCAL = KL > 0;
    for (;;) {
        const int s = __popcll(S);
        if (s <= a.dfs_max || uni < 0) {
            compact_dfs<KL>(A, S, H, P, h, p, lane, a, gs, vs, ct);
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
                if (LOCAL) P |= S;
                p += s;
                gs.leaf(h, p, lane, a.hist, a.hd);
                if (LOCAL) vs.leaf(h, p, H, P, lane, a);
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
            int slot = 0;
            if (lane == 0) slot = atomicAdd(a.c_out_n, nR);
            slot = bcast0(slot);
            if (slot + nR > a.c_cap) {
                if (lane == 0) atomicOr(a.flags, 1);
            } else if ((R >> lane) & 1) {
                const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
                CItem it;
                it.S = A & S & ~(R & below);
                it.H = H | (1ull << lane);
                it.P = P;
                it.uni = (uint32_t)uni;
                it.hp = (uint32_t)(h + 1) | ((uint32_t)p << 16);
                a.c_out[slot + __popcll(R & below)] = it;
            }
        }
        S &= Ap;
        if (LOCAL) P |= pbit;
        p++;
    }
    if (LOCAL) vs.flush(lane, nm, gid, root, pref, a);
}

// Write a compact universe (rows, member ids, prefix list); returns its
// index or -1 when the buffers are full.
template <int KL>
__device__ int make_universe(uint64_t A, int nm, int gid, int lane, const LevelArgs &a,
                             int root, uint64_t Hw, uint64_t Pw, const int *vl, int W,
                             int2 &pref) {
    constexpr bool LOCAL = KL > 0;
    int uni = 0;
    if (lane == 0) uni = atomicAdd(a.u_n, 1);
    uni = bcast0(uni);
    if (uni >= a.u_cap) {
        if (lane == 0) atomicOr(a.flags, 1);
        return -1;
    }
    a.u_rows[(long long)uni * 64 + lane] = (lane < nm) ? A : 0ull;
    pref = make_int2(0, 0);
    if (LOCAL) {
        a.u_gid[(long long)uni * 64 + lane] = (lane < nm) ? gid : -1;
        // prefix: the root plus the hold and pivot vertices above (word-major
        // multi-word sets Hw/Pw, lane w = word w)
        const int nh = (lane < W) ? __popcll(Hw) : 0, np = (lane < W) ? __popcll(Pw) : 0;
        const int tot = (int)wave_add_u32((uint32_t)(nh + np)) + 1;
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
                if ((hw >> lane) & 1) a.pref_pool[cur + __popcll(hw & below)] = vl[w * 64 + lane];
                cur += __popcll(hw);
                if ((pw >> lane) & 1)
                    a.pref_pool[cur + __popcll(pw & below)] = (int)(vl[w * 64 + lane] | 0x80000000u);
                cur += __popcll(pw);
            }
            pref = make_int2(off, tot);
            if (lane == 0) a.u_pref[uni] = pref;
        }
    }
    return uni;
}

// ---------------------------------------------------- multi-word tier
// Node sets over a heavy universe of up to 64*W vertices, lane w holding
// word w.  Rows are word-major in HBM: row u, word w at rows[w*dpad + u].

// Returns true with a compact start state (A, S0, nm, gid, uni, root,
// pref, h, p) once |S| <= 64, false if the buffers were full.
struct CState {
    uint64_t A, S, H, P;
    int h, p, uni, nm, gid, root;
    int2 pref;
};

template <int KL>
__device__ bool mw_run(int hu, uint64_t Sw, uint64_t Hw, uint64_t Pw, int h, int p, int lane,
                       const LevelArgs &a, Ctr &ct, int *memb, CState &cs) {
    constexpr bool LOCAL = KL > 0;
    const int W = a.W, dpad = a.dpad;
    const uint64_t *rows = a.hu_rows + (long long)hu * W * dpad;
    const int *vl = a.hu_vl + (long long)hu * dpad;
    const int root = a.order[a.heavy_base + hu];
    const bool wl = lane < W;
    if (!wl) Sw = Hw = Pw = 0;
    for (;;) {
        const int s = (int)wave_add_u32(wl ? (uint32_t)__popcll(Sw) : 0u);
        if (s <= 64) {
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
            uint64_t A = 0;
            for (int c = 0; c < s; c++) {
                const int mc = (int)readlane32((uint32_t)mj, c);
                bool bit = false;
                if (lane < s) bit = (rows[(long long)(mj >> 6) * dpad + mc] >> (mj & 63)) & 1;
                A = writelane64(A, ballot64(bit), c);
            }
            const int gid = (lane < s) ? vl[mj] : -1;
            int2 pref = make_int2(0, 0);
            int uni = -1;
            // the root and the multi-word holds/pivots form the prefix
            if (s > a.dfs_max || LOCAL) {
                uni = make_universe<KL>(A, s, gid, lane, a, root, Hw, Pw, vl, W, pref);
                if (uni < 0) return false;  // buffers full: the host reruns with larger ones
            }
            cs.A = A;
            cs.S = (s == 64) ? ~0ull : ((1ull << s) - 1);
            cs.H = cs.P = 0;
            cs.h = h;
            cs.p = p;
            cs.uni = (s > a.dfs_max) ? uni : -1;
            cs.nm = s;
            cs.gid = gid;
            cs.root = -1;
            cs.pref = pref;
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
                for (int w = 0; w < W; w++) c += (uint32_t)__popcll(rows[(long long)w * dpad + u] &
                                                                    readlane64(Sw, w));
                best = max(best, ((c + 1u) << 12) | (uint32_t)(4095 - u));
            }
        }
        best = wave_max_u32(best);
        const int piv = 4095 - (int)(best & 4095u);
        const int pc = (int)(best >> 12) - 1;
        const int pw = piv >> 6;
        const uint64_t pb = (lane == pw) ? (1ull << (piv & 63)) : 0ull;
        const uint64_t Ap = wl ? rows[(long long)lane * dpad + piv] : 0ull;
        if (pc + 1 != s && !(a.kmax > 0 && h + 1 > a.kmax)) {
            // hold children, increasing id, each N(S,v) minus earlier ones
            uint64_t Rw = Sw & ~Ap & ~pb;
            uint64_t Scur = Sw;
            const int nR = (int)wave_add_u32(wl ? (uint32_t)__popcll(Rw) : 0u);
            int slot = 0;
            if (lane == 0) slot = atomicAdd(a.mw_out_n, nR);
            slot = bcast0(slot);
            if (slot + nR > a.mw_cap) {
                if (lane == 0) atomicOr(a.flags, 1);
            } else {
                for (int i = 0; i < nR; i++) {
                    const uint64_t nzw = ballot64(wl && Rw != 0);
                    const int w0 = __builtin_ctzll(nzw);
                    const int v = w0 * 64 + __builtin_ctzll(readlane64(Rw, w0));
                    const uint64_t vb = (lane == w0) ? (1ull << (v & 63)) : 0ull;
                    uint64_t *it = a.mw_out + (long long)(slot + i) * a.mw_stride;
                    if (wl) {
                        it[lane] = rows[(long long)lane * dpad + v] & Scur;
                        it[W + lane] = Hw | vb;
                        it[2 * W + lane] = Pw;
                    }
                    if (lane == 0)
                        it[3 * W] = (uint64_t)(uint32_t)hu |
                                    ((uint64_t)((uint32_t)(h + 1) | ((uint32_t)p << 16)) << 32);
                    Scur &= ~vb;
                    Rw &= ~vb;
                }
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

__device__ uint64_t gather_light(int v, int lane, const LevelArgs &a, int *s_vl, int *s_pre,
                                 unsigned long long *s_A, int &d, int &gid) {
    const int b = a.orow[v];
    d = a.orow[v + 1] - b;
    const int u = (lane < d) ? a.ocol[b + lane] : 0x7fffffff;
    gid = (lane < d) ? u : -1;
    const int od = (lane < d) ? (a.orow[u + 1] - a.orow[u]) : 0;
    const int incl = wave_incl_scan(od);
    const int total = (int)readlane32((uint32_t)incl, 63);
    s_vl[lane] = u;
    s_pre[lane] = incl - od;
    s_A[lane] = 0ull;
    wave_sync();
    for (int q0 = 0; q0 < total; q0 += 64) {
        const int q = q0 + lane;
        if (q < total) {
            int lo = 0, hi = d - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_pre[mid] <= q) lo = mid; else hi = mid - 1;
            }
            const int j = lo;
            const int w = a.ocol[a.orow[s_vl[j]] + (q - s_pre[j])];
            int l2 = 0, h2 = d;
            while (l2 < h2) {
                const int mid = (l2 + h2) >> 1;
                if (s_vl[mid] < w) l2 = mid + 1; else h2 = mid;
            }
            if (l2 < d && s_vl[l2] == w) {
                atomicOr(&s_A[j], 1ull << l2);
                atomicOr(&s_A[l2], 1ull << j);
            }
        }
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

// --------------------------------------------------------- level kernel
// Work units of a level, in this order: multi-word items, compact items,
// and at level 0 the heavy roots then the light roots (largest first).

template <int KL>
__global__ void __launch_bounds__(64 * WAVES_PER_BLOCK) sct_level_kernel(const LevelArgs *__restrict__ pa) {
    constexpr bool LOCAL = KL > 0;
    const LevelArgs &a = *pa;
    __shared__ int s_vl[WAVES_PER_BLOCK][64];
    __shared__ int s_pre[WAVES_PER_BLOCK][64];
    __shared__ unsigned long long s_A[WAVES_PER_BLOCK][64];
    __shared__ int s_memb[WAVES_PER_BLOCK][64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    GlobalSink gs;
    gs.reset();
    gs.leaves = 0;
    VertexSink<KL> vs;
    if (LOCAL) vs.reset();
    Ctr ct;
    ct.nodes = ct.work = 0;

    const int n0 = a.n_mw_in, n1 = n0 + a.n_c_in;
    const int n2 = n1 + (a.level == 0 ? a.nheavy : 0);
    const int n3 = n2 + (a.level == 0 ? a.nlight : 0);
    for (;;) {
        int idx = 0;
        if (lane == 0) idx = atomicAdd(a.next, 1);
        idx = bcast0(__shfl(idx, 0, 64));
        if (idx >= n3) break;
        CState cs;
        bool run = true;
        if (idx < n0 || (idx >= n1 && idx < n2)) {
            // multi-word tier: an item of the previous level, or a heavy root
            int hu, h = 1, p = 0;
            uint64_t Sw = 0, Hw = 0, Pw = 0;
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
            } else {
                hu = idx - n1;
                const int v = a.order[a.heavy_base + hu];
                gather_heavy(hu, v, lane, a);
                const int d = a.orow[v + 1] - a.orow[v];
                // root node N+(v): every member; the root is the first hold vertex
                if (lane < a.W) {
                    const int cnt = min(max(d - lane * 64, 0), 64);
                    Sw = (cnt == 64) ? ~0ull : ((1ull << cnt) - 1);
                }
            }
            run = mw_run<KL>(hu, Sw, Hw, Pw, h, p, lane, a, ct, s_memb[wv], cs);
        } else if (idx < n1) {
            const CItem it = a.c_in[idx - n0];
            cs.A = a.u_rows[(long long)it.uni * 64 + lane];
            cs.S = it.S;
            cs.H = it.H;
            cs.P = it.P;
            cs.h = (int)(it.hp & 0xFFFFu);
            cs.p = (int)(it.hp >> 16);
            cs.uni = (int)it.uni;
            cs.gid = -1;
            cs.pref = make_int2(0, 0);
            if (LOCAL) {
                cs.gid = a.u_gid[(long long)it.uni * 64 + lane];
                cs.pref = a.u_pref[it.uni];
            }
            cs.nm = (int)wave_add_u32(cs.gid >= 0 ? 1u : 0u);
            cs.root = -1;
        } else {
            const int v = a.order[a.light_base + (idx - n2)];
            int d, gid;
            cs.A = gather_light(v, lane, a, s_vl[wv], s_pre[wv], s_A[wv], d, gid);
            cs.S = (d == 64) ? ~0ull : ((1ull << d) - 1);
            cs.H = cs.P = 0;
            cs.h = 1;
            cs.p = 0;
            cs.uni = -1;
            cs.nm = d;
            cs.gid = gid;
            cs.pref = make_int2(0, 0);
            if (d > a.dfs_max) {
                cs.uni = make_universe<KL>(cs.A, d, gid, lane, a, v, 0ull, 0ull, nullptr, 0, cs.pref);
                run = cs.uni >= 0;  // buffers full: the host reruns with larger ones
            }
            cs.root = (cs.uni < 0) ? v : -1;
        }
        if (run)
            compact_run<KL>(cs.A, cs.S, cs.H, cs.P, cs.h, cs.p, cs.uni, cs.nm, cs.gid, cs.root,
                            cs.pref, lane, a, gs, vs, ct);
    }
    gs.flush(lane, a.hist, a.hd);
    if (lane == 0) {
        atomicAdd(&a.counters[0], ct.nodes);
        atomicAdd(&a.counters[1], gs.leaves);
        atomicAdd(&a.counters[2], ct.work);
    }
}

// Roots with an empty out-neighbourhood are leaves (h=1, p=0) of the SCT.
__global__ void sct_sink_roots_kernel(int n, const int *__restrict__ order, const int *__restrict__ bounds,
                                      unsigned long long *hist, int hd, unsigned long long *counters,
                                      uint64_t *vout, int klo, int K) {
    const int first = bounds[1];
    const int cnt = n - first;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && cnt > 0) {
        atomicAdd(&hist[1 * hd + 0], (unsigned long long)cnt);
        atomicAdd(&counters[0], (unsigned long long)cnt);
        atomicAdd(&counters[1], (unsigned long long)cnt);
    }
    if (vout && klo == 1) {
        for (int j = i; j < cnt; j += gridDim.x * blockDim.x) {
            const int v = order[first + j];
            atomicAdd((unsigned long long *)(vout + 2 * ((long long)v * K)), 1ull);
        }
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

// ============================================================== host side

hipError_t pv_launch_level(const LevelArgs *a, int kl, int blocks, hipStream_t s) {
    if (kl == 0) sct_level_kernel<0><<<blocks, 64 * WAVES_PER_BLOCK, 0, s>>>(a);
    else if (kl <= 8) sct_level_kernel<8><<<blocks, 64 * WAVES_PER_BLOCK, 0, s>>>(a);
    else sct_level_kernel<16><<<blocks, 64 * WAVES_PER_BLOCK, 0, s>>>(a);
    return hipGetLastError();
}

int pv_level_blocks_per_cu(int kl) {
    int nb = 0;
    hipError_t e;
    if (kl == 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sct_level_kernel<0>, 64 * WAVES_PER_BLOCK, 0);
    else if (kl <= 8) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sct_level_kernel<8>, 64 * WAVES_PER_BLOCK, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sct_level_kernel<16>, 64 * WAVES_PER_BLOCK, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t pv_launch_sink_roots(int n, const int *order, const int *bounds, unsigned long long *hist,
                                int hd, unsigned long long *counters, uint64_t *vout, int klo, int K,
                                hipStream_t s) {
    sct_sink_roots_kernel<<<256, 256, 0, s>>>(n, order, bounds, hist, hd, counters, vout, klo, K);
    return hipGetLastError();
}

hipError_t pv_launch_binomials(int bn, uint64_t *tab128, uint8_t *bad, uint64_t *tab64, int *fits64,
                               hipStream_t s) {
    binom_kernel<<<1, 256, 0, s>>>(bn, tab128, bad, tab64, fits64);
    return hipGetLastError();
}

hipError_t pv_launch_finalize(const unsigned long long *hist, int hd, const uint64_t *tab128,
                              const uint8_t *bad, int bn, int kcap, int kmax, int c0,
                              uint64_t *counts, uint64_t *ovf_words, int *omega, hipStream_t s) {
    finalize_kernel<<<kcap, 256, 0, s>>>(hist, hd, tab128, bad, bn, kmax, c0, counts, ovf_words,
                                         omega);
    return hipGetLastError();
}
