// Degeneracy orientation on the GPU (Sec. 3, Lemma lem:degen; first step of
// Alg. 1).
//
// The paper removes a minimum-degree vertex at a time.  The parallel reading
// used here (the "canonical peel"): for level k = 0,1,..., in sub-rounds,
// remove *every* remaining vertex whose remaining degree is <= k, until none
// is left at that level.  A vertex's key is (sub-round, id); edges point from
// the smaller key to the larger, so every out-degree is at most the level at
// which the vertex left, and the largest level is the degeneracy alpha.
//
// One cooperative launch runs the whole peel.  The frontier of the next
// sub-round is exactly the set of vertices whose degree an atomic decrement
// takes from k+1 to k, so every vertex is appended once without rescanning
// the graph; only a level change scans the remaining vertices.  Sub-rounds
// end with a grid barrier while the graph is large (runs of sub-rounds with
// a handful of vertices each are taken by one workgroup between two grid
// barriers); its small remainder is finished by one workgroup (see below).
#include "common.h"
#include "internal.h"

#include <algorithm>

// ------------------------------------------------------------ validation
// Every row entry is checked: ids in range, no self loops, rows strictly
// increasing, and every (v,u) has its reverse (u,v), found by binary search
// in row u.  The entries are taken in chunks of VALIDATE_CHUNK, a wave per
// chunk, so a hub's row is spread over many waves; a lane finds the row of
// its entry by binary search of the row pointers between the rows of the
// chunk's first and last entries.  The row pointers are already checked
// (monotone, rp[0] = 0, rp[n] = nnz).
#define VALIDATE_CHUNK 512

// the row holding entry i: the largest v in [lo, hi] with rp[v] <= i
__device__ __forceinline__ int row_of(const int *__restrict__ rp, int lo, int hi, int i) {
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rp[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(256) validate_kernel(int n, int nnz, const int *__restrict__ rp,
                                                        const int *__restrict__ col,
                                                        int *__restrict__ err) {
    const int lane = threadIdx.x & 63;
    const long long nw = (long long)(gridDim.x * blockDim.x) >> 6;
    bool bad = false;
    for (long long c0 = (long long)((blockIdx.x * blockDim.x + threadIdx.x) >> 6) * VALIDATE_CHUNK; c0 < nnz;
         c0 += nw * VALIDATE_CHUNK) {
        const int i0 = (int)c0, i1 = (int)min(c0 + VALIDATE_CHUNK, (long long)nnz) - 1;
        // rows of the chunk's first and last entries (lanes 0 and 1)
        int r = 0;
        if (lane < 2) r = row_of(rp, 0, n - 1, lane == 0 ? i0 : i1);
        const int va = __shfl(r, 0), vb = __shfl(r, 1);
        for (int i = i0 + lane; i <= i1; i += 64) {
            const int v = (va == vb) ? va : row_of(rp, va, vb, i);
            const int u = col[i];
            if (u < 0 || u >= n || u == v) {
                bad = true;
                continue;
            }
            if (i > rp[v] && col[i - 1] >= u) bad = true;
            int lo = rp[u], hi = rp[u + 1];
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (col[mid] < v) lo = mid + 1; else hi = mid;
            }
            if (lo >= rp[u + 1] || col[lo] != v) bad = true;
        }
    }
    if (ballot64(bad) && lane == 0) atomicOr(err, 2);
}

__global__ void check_rowptr_kernel(int n, long long nnz, const int *__restrict__ rp,
                                    int *__restrict__ err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && (rp[0] != 0 || (long long)rp[n] != nnz)) atomicOr(err, 1);
    if (i < n && rp[i + 1] < rp[i]) atomicOr(err, 1);
}

// ------------------------------------------------------------------ peel
// Grid-wide phase: while more than PV_SOLO_MAX vertices remain, every block
// takes part and a sub-round ends with a grid barrier.  Solo phase: the
// remaining subgraph is compacted (local ids, local CSR of the edges among
// the remaining vertices) and block 0 finishes the peel alone with its
// degrees and frontiers in LDS and block-level barriers.  Both phases run
// the same sub-rounds, so the keys are those of the canonical peel.

// a relaxed device-scope load (no ordering of its own: where a value read
// this way publishes other data, a fence after it gives the acquire)
__device__ __forceinline__ int ld_agent_rlx(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned ld_u(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier for a launch whose blocks are all resident at once.  Every block
// publishes the number of barriers it has passed on its own 128-byte line
// (a release store; `epoch` is that number, kept by the caller), and one
// wave of each block polls all the lines until every block has reached the
// same barrier: no chain of read-modify-writes, one round trip after the
// last arrival.  A bounded wait turns a lost block into an error flag
// instead of a hang; returns false then.
__device__ bool grid_barrier(PeelCtl *ctl, int nblocks, unsigned &epoch) {
    __syncthreads();
    __shared__ int s_ok;
    const unsigned e = ++epoch;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        if (lane == 0) {
            __threadfence();
            __hip_atomic_store(&ctl->bar_flag[blockIdx.x * 32], e, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        int ok = 1;
        unsigned spins = 0;
        for (;;) {
            bool behind = false;
            for (int b = lane; b < nblocks; b += 64) behind = behind || ld_u(&ctl->bar_flag[b * 32]) < e;
            if (ballot64(behind) == 0) break;
            if (ld_agent_rlx(&ctl->err) != 0 || ++spins > (1u << 24)) {
                if (lane == 0) atomicOr(&ctl->err, 1);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __threadfence();
        if (lane == 0) s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// edges a wave takes per step of a frontier vertex's row (4 per lane, so
// that four independent load/atomic chains are in flight)
#define PEEL_UNROLL 4
// frontier rows of at most this many entries are walked one per lane
#define PEEL_LANE_ROW 32
// joins a block gathers in LDS per sub-round before the rest go straight to
// the next frontier
#define PEEL_JOIN_LDS 4096
// vertices per thread a level change reads with their loads in flight
// together (and holds in registers when one batch covers the graph)
#define PEEL_LC_BATCH 16
// vertices per thread whose loads a level change's take pass has in flight
// together when the degrees are read again (fewer than PEEL_LC_BATCH: the
// take keeps three values per vertex live)
#define PEEL_TAKE_BATCH 8
// row entries per lane a step of U's compaction reads (loads in flight)
#define PEEL_CSR_UNROLL 8
// rows of U longer than this are split over the grid's waves
#define PEEL_LONG_ROW 4096
// frontiers of at most this many vertices are removed by block 0 alone, up
// to PEEL_BLOCK_ROUNDS sub-rounds in a row between two grid barriers
#define PEEL_BLOCK_FRONTIER 32
#define PEEL_BLOCK_ROUNDS 256
// local vertices per thread in the solo phase (blockDim.x == PV_PEEL_THREADS)
#define PEEL_SOLO_PER_THREAD (PV_SOLO_MAX / PV_PEEL_THREADS)
static_assert(PV_SOLO_MAX % PV_PEEL_THREADS == 0, "solo phase: whole vertices per thread");

// exclusive prefix sum over the block (blockDim.x == PV_PEEL_THREADS);
// returns the block total in *total
__device__ int block_excl_scan(int x, int *total) {
    __shared__ int s_w[PV_PEEL_THREADS / 64 + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int inc = wave_incl_scan(x);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < PV_PEEL_THREADS / 64; i++) {
            const int t = s_w[i];
            s_w[i] = acc;
            acc += t;
        }
        s_w[PV_PEEL_THREADS / 64] = acc;
    }
    __syncthreads();
    const int r = s_w[w] + inc - x;
    *total = s_w[PV_PEEL_THREADS / 64];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(PV_PEEL_THREADS) peel_kernel(PeelArgs pa) {
    const int n = pa.n;
    const int *__restrict__ rp = pa.rp;
    const int *__restrict__ col = pa.col;
    int *__restrict__ deg = pa.deg;
    int *__restrict__ sub = pa.sub;
    PeelCtl *__restrict__ ctl = pa.ctl;
    const int nb = gridDim.x;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nth = gridDim.x * blockDim.x;
    const int lane = threadIdx.x & 63;
    const int wid = tid >> 6;
    const int nw = nth >> 6;

    unsigned epoch = 0;  // grid barriers this block has passed
    if (tid == 0) ctl->t_mark[0] = __builtin_amdgcn_s_memrealtime();
    int n_grid = 0, n_block = 0, n_levels = 0;  // kept by block 0 for the diagnostics
    for (int v = tid; v < n; v += nth) {
        deg[v] = rp[v + 1] - rp[v];
        sub[v] = -1;
    }
    if (!grid_barrier(ctl, nb, epoch)) return;

    // ---------------------------------------------------- grid-wide phase
    // vertices a block appends to a frontier are gathered in LDS and moved
    // with one global atomic per block (a counter taken by every wave
    // serialises across the XCDs); past the LDS list's end they go straight
    // to the frontier.  s_nj is zero when a list starts (the caller's
    // barrier orders the reset); list_flush ends with the block's copies
    // done.
    __shared__ int s_join[PEEL_JOIN_LDS];
    __shared__ int s_nj, s_jbase, s_kmin;
    // a wave holding list slots [slot, slot + cnt_) sends those past the LDS
    // list's end straight to the frontier, reserved with one global atomic
    // for the wave (one per vertex serialises on the counter: 1.6M vertices
    // of a first level took 21 ms); entry sl >= PEEL_JOIN_LDS goes to
    // Fo[base + sl - first]
    const auto overflow_base = [&](int slot, int cnt_, int *cnt) {
        const int first = max(slot, PEEL_JOIN_LDS);
        const int over = slot + cnt_ - first;
        int base = 0;
        if (over > 0 && lane == 0) base = atomicAdd(cnt, over);
        return __shfl(base, 0) - first;
    };
    const auto list_flush = [&](int *Fo, int *cnt) {
        __syncthreads();
        const int nj = min(s_nj, PEEL_JOIN_LDS);
        if (threadIdx.x == 0) s_jbase = nj ? atomicAdd(cnt, nj) : 0;
        __syncthreads();
        for (int j = threadIdx.x; j < nj; j += blockDim.x) Fo[s_jbase + j] = s_join[j];
    };
    int removed = 0, r = 0, k = 0, nF = 0, alpha = 0;
    while (n - removed > PV_SOLO_MAX) {
        if (nF == 0) {
            // level change: k = smallest remaining degree (a block minimum
            // in LDS, one global atomic per block).  A thread reads its
            // vertices tid, tid + nth, ... PEEL_LC_BATCH at a time with all
            // loads in flight together; when one batch covers the graph, the
            // degrees stay in registers for the take pass (no decrement
            // happens between the two passes).
            n_levels++;
            if (threadIdx.x == 0) s_kmin = 0x7fffffff;
            __syncthreads();
            int mymin = 0x7fffffff;
            int dk[PEEL_LC_BATCH];  // remaining degree; INT_MAX if removed or past n
#pragma unroll
            for (int q = 0; q < PEEL_LC_BATCH; q++) dk[q] = 0x7fffffff;
            for (int v0 = tid; v0 < n; v0 += nth * PEEL_LC_BATCH) {
                int sq[PEEL_LC_BATCH];
#pragma unroll
                for (int q = 0; q < PEEL_LC_BATCH; q++) {
                    const int v = v0 + q * nth < n ? v0 + q * nth : 0;
                    sq[q] = sub[v];
                    dk[q] = deg[v];
                }
#pragma unroll
                for (int q = 0; q < PEEL_LC_BATCH; q++) {
                    if (v0 + q * nth >= n || sq[q] >= 0) dk[q] = 0x7fffffff;
                    mymin = min(mymin, dk[q]);
                }
            }
            const bool held = n <= nth * PEEL_LC_BATCH;
            mymin = wave_min_i32(mymin);
            if (lane == 0) atomicMin(&s_kmin, mymin);
            __syncthreads();
            if (threadIdx.x == 0 && s_kmin != 0x7fffffff) atomicMin(&ctl->minv[r & 1], s_kmin);
            if (!grid_barrier(ctl, nb, epoch)) return;
            k = ld_agent_rlx(&ctl->minv[r & 1]);
            alpha = max(alpha, k);
            int *F = (r & 1) ? pa.fb : pa.fa;
            if (threadIdx.x == 0) s_nj = 0;
            __syncthreads();
            if (held) {
                // vertex tid + q * nth is this lane's q-th (dk is INT_MAX
                // past n); a wave reserves the list slots of all its takes
                // with one LDS atomic
                int tt = 0;
#pragma unroll
                for (int q = 0; q < PEEL_LC_BATCH; q++) tt += __popcll(ballot64(dk[q] <= k));
                if (tt) {
                    const uint64_t bl = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
                    int slot = 0;
                    if (lane == 0) slot = atomicAdd(&s_nj, tt);
                    slot = __shfl(slot, 0);
                    const int ob = overflow_base(slot, tt, &ctl->cnt[r % 3]);
#pragma unroll
                    for (int q = 0; q < PEEL_LC_BATCH; q++) {
                        const bool take = dk[q] <= k;
                        const uint64_t m = ballot64(take);
                        if (take) {
                            const int v = tid + q * nth;
                            sub[v] = r;
                            const int sl = slot + __popcll(m & bl);
                            if (sl < PEEL_JOIN_LDS) s_join[sl] = v;
                            else F[ob + sl] = v;
                        }
                        slot += __popcll(m);
                    }
                }
            } else {
                // the same take, reading the degrees again: PEEL_TAKE_BATCH
                // vertices per thread with their loads in flight together
                // (a pass of one vertex per lane waits on a load pair per
                // 64 vertices of a wave: 64 round trips per level change on
                // a 4M-vertex graph)
                const uint64_t bl = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
                for (int vb = 0; vb < n; vb += nth * PEEL_TAKE_BATCH) {
                    bool tk[PEEL_TAKE_BATCH];
                    int sq[PEEL_TAKE_BATCH], dq[PEEL_TAKE_BATCH];
#pragma unroll
                    for (int q = 0; q < PEEL_TAKE_BATCH; q++) {
                        const int v = vb + q * nth + tid;
                        const int vv = v < n ? v : 0;
                        sq[q] = sub[vv];
                        dq[q] = deg[vv];
                    }
                    int tt = 0;
#pragma unroll
                    for (int q = 0; q < PEEL_TAKE_BATCH; q++) {
                        tk[q] = vb + q * nth + tid < n && sq[q] < 0 && dq[q] <= k;
                        tt += __popcll(ballot64(tk[q]));
                    }
                    if (tt) {
                        int slot = 0;
                        if (lane == 0) slot = atomicAdd(&s_nj, tt);
                        slot = __shfl(slot, 0);
                        const int ob = overflow_base(slot, tt, &ctl->cnt[r % 3]);
#pragma unroll
                        for (int q = 0; q < PEEL_TAKE_BATCH; q++) {
                            const uint64_t m = ballot64(tk[q]);
                            if (tk[q]) {
                                const int v = vb + q * nth + tid;
                                sub[v] = r;
                                const int sl = slot + __popcll(m & bl);
                                if (sl < PEEL_JOIN_LDS) s_join[sl] = v;
                                else F[ob + sl] = v;
                            }
                            slot += __popcll(m);
                        }
                    }
                }
            }
            list_flush(F, &ctl->cnt[r % 3]);
            if (!grid_barrier(ctl, nb, epoch)) return;
            nF = ld_agent_rlx(&ctl->cnt[r % 3]);
            if (nF == 0) break;  // cannot happen while vertices remain
        }
        const int *F = (r & 1) ? pa.fb : pa.fa;
        int *Fn = (r & 1) ? pa.fa : pa.fb;
        if (tid == 0) {
            ctl->cnt[(r + 2) % 3] = 0;
            ctl->minv[(r + 1) & 1] = 0x7fffffff;
        }
        // remove the frontier: decrement the degrees of remaining neighbours;
        // a neighbour taken from k+1 to k joins the next sub-round
        int *ncnt = &ctl->cnt[(r + 1) % 3];
        // joins of this sub-round: the block's LDS list
        if (threadIdx.x == 0) s_nj = 0;
        __syncthreads();
        // one decrement per remaining neighbour; a neighbour taken from k+1
        // to k joins the next sub-round (appended, one atomic per wave)
        const auto visit = [&](const int (&u)[PEEL_UNROLL], bool (&live)[PEEL_UNROLL]) {
#pragma unroll
            for (int q = 0; q < PEEL_UNROLL; q++)
                live[q] = live[q] &&
                          __hip_atomic_load(&sub[u[q]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < 0;
            int old[PEEL_UNROLL];
#pragma unroll
            for (int q = 0; q < PEEL_UNROLL; q++) old[q] = live[q] ? atomicSub(&deg[u[q]], 1) : 0;
            // one slot reservation in the block's list for all the joins
            bool join[PEEL_UNROLL];
            uint64_t jm[PEEL_UNROLL];
            int jt = 0;
#pragma unroll
            for (int q = 0; q < PEEL_UNROLL; q++) {
                join[q] = live[q] && old[q] == k + 1;
                if (join[q]) sub[u[q]] = r + 1;
                jm[q] = ballot64(join[q]);
                jt += __popcll(jm[q]);
            }
            if (jt) {
                const uint64_t bl = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
                int slot = 0;
                if (lane == 0) slot = atomicAdd(&s_nj, jt);
                slot = __shfl(slot, 0);
                const int ob = overflow_base(slot, jt, ncnt);
#pragma unroll
                for (int q = 0; q < PEEL_UNROLL; q++) {
                    if (join[q]) {
                        const int sl = slot + __popcll(jm[q] & bl);
                        if (sl < PEEL_JOIN_LDS) s_join[sl] = u[q];
                        else Fn[ob + sl] = u[q];
                    }
                    slot += __popcll(jm[q]);
                }
            }
        };
        // a row walked by the whole wave, 64 * PEEL_UNROLL entries at a time
        const auto wave_row = [&](int w0, int w1) {
            for (int eb = w0; eb < w1; eb += 64 * PEEL_UNROLL) {
                int u[PEEL_UNROLL];
                bool live[PEEL_UNROLL];
#pragma unroll
                for (int q = 0; q < PEEL_UNROLL; q++) {
                    const int e = eb + q * 64 + lane;
                    live[q] = e < w1;
                    u[q] = col[live[q] ? e : w0];
                }
                visit(u, live);
            }
        };
        if (nF <= PEEL_BLOCK_FRONTIER) {
            // a small frontier (the tail of a level): block 0 runs this
            // sub-round and the next small ones alone, one wave per frontier
            // vertex and workgroup barriers only, while the other blocks
            // wait at the next grid barrier.  Within the block, frontiers
            // are read back with agent-scope loads (never a stale L1 line);
            // removal keys and degrees already go through atomics.  The grid
            // barrier then publishes everything, and where block 0 stopped.
            if (blockIdx.x == 0) {
                const int bw = threadIdx.x >> 6, nbw = blockDim.x >> 6;
                for (int t = 0;; t++) {
                    for (int i = bw; i < nF; i += nbw) {
                        const int v = ld_agent_rlx(&F[i]);
                        wave_row(rp[v], rp[v + 1]);
                    }
                    list_flush(Fn, ncnt);
                    __syncthreads();
                    removed += nF;
                    nF = ld_agent_rlx(ncnt);
                    r++;
                    n_block++;
                    if (nF == 0 || nF > PEEL_BLOCK_FRONTIER || t + 1 >= PEEL_BLOCK_ROUNDS ||
                        n - removed <= PV_SOLO_MAX)
                        break;
                    F = (r & 1) ? pa.fb : pa.fa;
                    Fn = (r & 1) ? pa.fa : pa.fb;
                    ncnt = &ctl->cnt[(r + 1) % 3];
                    if (threadIdx.x == 0) {
                        ctl->cnt[(r + 2) % 3] = 0;
                        ctl->minv[(r + 1) & 1] = 0x7fffffff;
                        s_nj = 0;
                    }
                    __syncthreads();
                }
                if (threadIdx.x == 0) {
                    ctl->blk_r = r;
                    ctl->blk_nf = nF;
                    ctl->blk_removed = removed;
                }
            }
            if (!grid_barrier(ctl, nb, epoch)) return;
            r = ld_agent_rlx(&ctl->blk_r);
            nF = ld_agent_rlx(&ctl->blk_nf);
            removed = ld_agent_rlx(&ctl->blk_removed);
            continue;
        }
        if (nF >= nw * 8) {
            // a large frontier (the first sub-rounds of the low levels): a
            // wave takes 64 vertices at a time, vertex i0 + lane * nw + wid
            // in lane `lane`; rows of at most PEEL_LANE_ROW entries are
            // walked one per lane, longer ones by the whole wave
            for (int i0 = 0; i0 < nF; i0 += nw * 64) {
                const int i = i0 + lane * nw + wid;
                int v = 0, e0 = 0, e1 = 0;
                if (i < nF) {
                    v = F[i];
                    e0 = rp[v];
                    e1 = rp[v + 1];
                }
                const bool wide = i < nF && e1 - e0 > PEEL_LANE_ROW;
                const int end = (i < nF && !wide) ? e1 : 0;
                for (int e = (i < nF && !wide) ? e0 : 0; ballot64(e < end); e += PEEL_UNROLL) {
                    int u[PEEL_UNROLL];
                    bool live[PEEL_UNROLL];
#pragma unroll
                    for (int q = 0; q < PEEL_UNROLL; q++) {
                        live[q] = e + q < end;
                        u[q] = live[q] ? col[e + q] : 0;
                    }
                    visit(u, live);
                }
                for (uint64_t wm = ballot64(wide); wm; wm &= wm - 1ull) {
                    const int vv = __shfl(v, __builtin_ctzll(wm), 64);
                    wave_row(rp[vv], rp[vv + 1]);
                }
            }
        } else {
            for (int i = wid; i < nF; i += nw) {
                const int v = F[i];
                wave_row(rp[v], rp[v + 1]);
            }
        }
        list_flush(Fn, ncnt);
        if (!grid_barrier(ctl, nb, epoch)) return;
        removed += nF;
        nF = ld_agent_rlx(&ctl->cnt[(r + 1) % 3]);
        r++;
        n_grid++;
    }
    if (tid == 0) {
        ctl->t_mark[1] = __builtin_amdgcn_s_memrealtime();
        ctl->n_grid = n_grid;
        ctl->n_block = n_block;
        ctl->n_levels = n_levels;
        ctl->n_solo = n - removed;
    }

    // ------------------------------------ compaction of what is left (U)
    // U = remaining vertices plus the pending frontier (keys of the pending
    // frontier are already r; its decrements are still to be done).
    __shared__ int s_off;
    const int chunk = (n + nb - 1) / nb;
    const int lo = min(n, blockIdx.x * chunk), hi = min(n, lo + chunk);
    {
        int cnt = 0;
        for (int v = lo + threadIdx.x; v < hi; v += blockDim.x) {
            const int s = sub[v];
            cnt += (s < 0 || s == r) ? 1 : 0;
        }
        int tot;
        (void)block_excl_scan(cnt, &tot);
        if (threadIdx.x == 0) pa.bcnt[blockIdx.x] = tot;
    }
    if (!grid_barrier(ctl, nb, epoch)) return;
    if (threadIdx.x == 0) {
        int off = 0;
        for (int b = 0; b < (int)blockIdx.x; b++) off += pa.bcnt[b];
        s_off = off;
    }
    __syncthreads();
    {
        int base = s_off;
        for (int v0 = lo; v0 < hi; v0 += blockDim.x) {
            const int v = v0 + threadIdx.x;
            bool inU = false;
            if (v < hi) {
                const int s = sub[v];
                inU = (s < 0 || s == r);
            }
            int tot;
            const int pos = block_excl_scan(inU ? 1 : 0, &tot);
            if (v < hi) {
                pa.lid[v] = inU ? base + pos : -1;
                if (inU) pa.uverts[base + pos] = v;
            }
            base += tot;
        }
    }
    if (!grid_barrier(ctl, nb, epoch)) return;
    const int nu = n - removed;
    if (nu > PV_SOLO_MAX) {  // only if the grid phase stopped early: report, never overflow
        if (threadIdx.x == 0) atomicOr(&ctl->err, 2);
        return;
    }
    // induced degree of every vertex of U and its local CSR: neighbours
    // inside U, as local ids.  A wave reads 64 * PEEL_CSR_UNROLL entries of
    // a row a step with the loads in flight together.  Rows longer than
    // PEEL_LONG_ROW (the hubs, on U's critical path) are listed in
    // pa.lrow and split over the grid's waves: G = nw / nl waves per row,
    // each taking every G-th step of it; their degrees are summed with
    // atomics and their CSR entries placed through a cursor per row, in no
    // particular order (the solo phase does not depend on the order within
    // a row).  Other rows keep their row order.
    const auto row_step = [&](int eb, int e0, int e1, int (&l)[PEEL_CSR_UNROLL]) {
#pragma unroll
        for (int q = 0; q < PEEL_CSR_UNROLL; q++) {
            const int e = eb + q * 64 + lane;
            l[q] = col[e < e1 ? e : e0];
        }
#pragma unroll
        for (int q = 0; q < PEEL_CSR_UNROLL; q++) l[q] = pa.lid[l[q]];
#pragma unroll
        for (int q = 0; q < PEEL_CSR_UNROLL; q++)
            if (eb + q * 64 + lane >= e1) l[q] = -1;
    };
    constexpr int SEG = 64 * PEEL_CSR_UNROLL;
    for (int i = wid; i < nu; i += nw) {
        const int v = pa.uverts[i];
        const int e0 = rp[v], e1 = rp[v + 1];
        if (e1 - e0 > PEEL_LONG_ROW) {
            if (lane == 0) {
                pa.lrow[atomicAdd(&ctl->nlong, 1)] = i;  // at most nu <= PV_SOLO_MAX rows
                pa.ldeg[i] = 0;
            }
            continue;
        }
        int c = 0;
        for (int eb = e0; eb < e1; eb += SEG) {
            int l[PEEL_CSR_UNROLL];
            row_step(eb, e0, e1, l);
#pragma unroll
            for (int q = 0; q < PEEL_CSR_UNROLL; q++) c += l[q] >= 0 ? 1 : 0;
        }
        c = (int)wave_add_u32((uint32_t)c);
        if (lane == 0) pa.ldeg[i] = c;
    }
    if (!grid_barrier(ctl, nb, epoch)) return;
    const int nl = ld_agent_rlx(&ctl->nlong);
    const int G = nl > 0 ? max(1, nw / nl) : 1;
    // long rows: wave t takes row t % nl from step t / nl on, every G-th step
    for (int t = wid; t < nl * G; t += nw) {
        const int i = pa.lrow[t % nl];
        const int v = pa.uverts[i];
        const int e0 = rp[v], e1 = rp[v + 1];
        int c = 0;
        for (int eb = e0 + (t / nl) * SEG; eb < e1; eb += G * SEG) {
            int l[PEEL_CSR_UNROLL];
            row_step(eb, e0, e1, l);
#pragma unroll
            for (int q = 0; q < PEEL_CSR_UNROLL; q++) c += l[q] >= 0 ? 1 : 0;
        }
        c = (int)wave_add_u32((uint32_t)c);
        if (lane == 0 && c) atomicAdd(&pa.ldeg[i], c);
    }
    if (!grid_barrier(ctl, nb, epoch)) return;
    if (blockIdx.x == 0) {
        int base = 0;
        for (int i0 = 0; i0 < nu; i0 += blockDim.x) {
            const int i = i0 + threadIdx.x;
            const int x = (i < nu) ? pa.ldeg[i] : 0;
            int tot;
            const int pos = block_excl_scan(x, &tot);
            if (i < nu) pa.lrp[i] = base + pos;
            base += tot;
        }
        if (threadIdx.x == 0) pa.lrp[nu] = base;
        __syncthreads();
        // fill cursor of every long row: its row start
        for (int j = threadIdx.x; j < nl; j += blockDim.x) pa.lrow[PV_SOLO_MAX + j] = pa.lrp[pa.lrow[j]];
    }
    if (!grid_barrier(ctl, nb, epoch)) return;
    {
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        for (int i = wid; i < nu; i += nw) {
            const int v = pa.uverts[i];
            const int e0 = rp[v], e1 = rp[v + 1];
            if (e1 - e0 > PEEL_LONG_ROW) continue;
            int w = pa.lrp[i];
            for (int eb = e0; eb < e1; eb += SEG) {
                int l[PEEL_CSR_UNROLL];
                row_step(eb, e0, e1, l);
#pragma unroll
                for (int q = 0; q < PEEL_CSR_UNROLL; q++) {
                    const uint64_t m = ballot64(l[q] >= 0);
                    if (l[q] >= 0) pa.lcol[w + __popcll(m & below)] = l[q];
                    w += __popcll(m);
                }
            }
        }
        for (int t = wid; t < nl * G; t += nw) {
            const int j = t % nl;
            const int v = pa.uverts[pa.lrow[j]];
            const int e0 = rp[v], e1 = rp[v + 1];
            for (int eb = e0 + (t / nl) * SEG; eb < e1; eb += G * SEG) {
                int l[PEEL_CSR_UNROLL];
                row_step(eb, e0, e1, l);
                uint64_t m[PEEL_CSR_UNROLL];
                int tot = 0;
#pragma unroll
                for (int q = 0; q < PEEL_CSR_UNROLL; q++) {
                    m[q] = ballot64(l[q] >= 0);
                    tot += __popcll(m[q]);
                }
                if (tot == 0) continue;
                int w = 0;
                if (lane == 0) w = atomicAdd(&pa.lrow[PV_SOLO_MAX + j], tot);
                w = __shfl(w, 0);
#pragma unroll
                for (int q = 0; q < PEEL_CSR_UNROLL; q++) {
                    if (l[q] >= 0) pa.lcol[w + __popcll(m[q] & below)] = l[q];
                    w += __popcll(m[q]);
                }
            }
        }
    }
    if (!grid_barrier(ctl, nb, epoch)) return;
    if (blockIdx.x != 0) return;
    if (threadIdx.x == 0) ctl->t_mark[2] = __builtin_amdgcn_s_memrealtime();

    // ------------------------------------------------ solo phase (block 0)
    // LDS holds the remaining degrees as 16-bit halves of 32-bit words (a
    // degree only counts neighbours still in U and is decremented at most
    // once per neighbour, so a half never borrows from the other), liveness
    // as a bitmask, the local row offsets, and the frontiers as 16-bit local
    // ids, one after the other (every vertex joins one frontier, so all fit
    // in PV_SOLO_MAX entries).  A removed vertex's degree half is not read
    // again: once its sub-round's decrements are over (after the barrier)
    // it holds the vertex's sub-round minus r0, and one pass at the end
    // writes the keys.
    __shared__ unsigned s_deg2[PV_SOLO_MAX / 2];
    __shared__ unsigned s_alive[PV_SOLO_MAX / 32];
    __shared__ unsigned short s_Fq[PV_SOLO_MAX];
    __shared__ int s_lrp[PV_SOLO_MAX + 1];
    // s_cnt3[(r + 1) % 3] counts the joins of sub-round r; the next but one
    // is reset while r runs, so the counters need no barrier of their own
    __shared__ int s_cnt3[3], s_min;
    unsigned short *const s_h16 = (unsigned short *)s_deg2;  // half i = vertex i
    const int *__restrict__ lcol = pa.lcol;
    const int *__restrict__ uverts = pa.uverts;
    const int r0 = r;
    if (threadIdx.x < 3) s_cnt3[threadIdx.x] = 0;
    for (int i = threadIdx.x; i < PV_SOLO_MAX / 32; i += blockDim.x) s_alive[i] = 0u;
    for (int i = threadIdx.x; i <= nu; i += blockDim.x) s_lrp[i] = pa.lrp[i];
    __syncthreads();
    for (int i = threadIdx.x; i < (nu + 1) / 2; i += blockDim.x) {
        const int a = 2 * i, b = 2 * i + 1;
        const unsigned lo = (unsigned)pa.ldeg[a] & 0xFFFFu;
        const unsigned hi = (b < nu) ? ((unsigned)pa.ldeg[b] & 0xFFFFu) : 0u;
        s_deg2[i] = lo | (hi << 16);
    }
    for (int i = threadIdx.x; i < nu; i += blockDim.x)
        if (sub[uverts[i]] < 0) atomicOr(&s_alive[i >> 5], 1u << (i & 31));
    __syncthreads();
    auto alive = [&](int i) -> bool { return (s_alive[i >> 5] >> (i & 31)) & 1u; };
    auto degof = [&](int i) -> int { return (int)s_h16[i]; };
    int fbase = 0;  // the current frontier is s_Fq[fbase, fbase + nF)
    if (nF > 0) {
        // the pending frontier of the grid phase (its sub-round is r0)
        const int *F = (r & 1) ? pa.fb : pa.fa;
        for (int j = threadIdx.x; j < nF; j += blockDim.x) s_Fq[j] = (unsigned short)pa.lid[F[j]];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nF; j += blockDim.x) s_h16[s_Fq[j]] = 0;
    __syncthreads();
    const int bw = threadIdx.x >> 6, nbw = blockDim.x >> 6;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int left = nu;
    for (;;) {
        if (nF == 0) {
            if (left == 0) break;
            // level change: local vertex threadIdx.x + q * blockDim.x is
            // this thread's q-th; its remaining degree (INT_MAX once removed)
            // stays in a register from the minimum to the take, and a wave
            // reserves the slots of all its takes with one LDS atomic
            if (threadIdx.x == 0) s_min = 0x7fffffff;
            __syncthreads();
            int dq[PEEL_SOLO_PER_THREAD];
            int mymin = 0x7fffffff;
#pragma unroll
            for (int q = 0; q < PEEL_SOLO_PER_THREAD; q++) {
                const int i = threadIdx.x + q * PV_PEEL_THREADS;
                dq[q] = (i < nu && alive(i)) ? degof(i) : 0x7fffffff;
                mymin = min(mymin, dq[q]);
            }
            mymin = wave_min_i32(mymin);
            if (lane == 0) atomicMin(&s_min, mymin);
            __syncthreads();
            k = s_min;
            alpha = max(alpha, k);
            // the frontier of sub-round r, counted on s_cnt3[r % 3]
            if (threadIdx.x == 0) s_cnt3[r % 3] = 0;
            __syncthreads();
            int tt = 0;
#pragma unroll
            for (int q = 0; q < PEEL_SOLO_PER_THREAD; q++) tt += __popcll(ballot64(dq[q] <= k));
            if (tt) {
                int slot = 0;
                if (lane == 0) slot = atomicAdd(&s_cnt3[r % 3], tt);
                slot = fbase + __shfl(slot, 0);
#pragma unroll
                for (int q = 0; q < PEEL_SOLO_PER_THREAD; q++) {
                    const int i = threadIdx.x + q * PV_PEEL_THREADS;
                    const bool take = dq[q] <= k;
                    const uint64_t m = ballot64(take);
                    if (take) {
                        atomicAnd(&s_alive[i >> 5], ~(1u << (i & 31)));
                        s_Fq[slot + __popcll(m & below)] = (unsigned short)i;
                    }
                    slot += __popcll(m);
                }
            }
            __syncthreads();
            nF = s_cnt3[r % 3];
            if (nF == 0) break;
            // (a removed vertex's half is not read again; its 16-bit store
            // leaves the other half of the word, which decrements may still
            // change, untouched)
            for (int j = threadIdx.x; j < nF; j += blockDim.x) s_h16[s_Fq[fbase + j]] = (unsigned short)(r - r0);
        }
        if (threadIdx.x == 0) s_cnt3[(r + 2) % 3] = 0;
        // joins are appended after the current frontier
        const int nbase = fbase + nF;
        for (int j = bw; j < nF; j += nbw) {
            const int i = s_Fq[fbase + j];
            const int e0 = s_lrp[i], e1 = s_lrp[i + 1];
            for (int eb = e0; eb < e1; eb += 64 * PEEL_UNROLL) {
                int w[PEEL_UNROLL];
                bool live[PEEL_UNROLL];
#pragma unroll
                for (int q = 0; q < PEEL_UNROLL; q++) {
                    const int e = eb + q * 64 + lane;
                    live[q] = e < e1;
                    w[q] = lcol[live[q] ? e : e0];
                }
                // the step's decrements first, then one slot reservation for
                // all its joins
                bool join[PEEL_UNROLL];
#pragma unroll
                for (int q = 0; q < PEEL_UNROLL; q++) {
                    join[q] = false;
                    if (live[q] && alive(w[q])) {
                        const unsigned sh = (w[q] & 1) * 16;
                        const unsigned old = atomicSub(&s_deg2[w[q] >> 1], 1u << sh);
                        if ((int)((old >> sh) & 0xFFFFu) == k + 1) {
                            atomicAnd(&s_alive[w[q] >> 5], ~(1u << (w[q] & 31)));
                            join[q] = true;
                        }
                    }
                }
                uint64_t jm[PEEL_UNROLL];
                int jt = 0;
#pragma unroll
                for (int q = 0; q < PEEL_UNROLL; q++) {
                    jm[q] = ballot64(join[q]);
                    jt += __popcll(jm[q]);
                }
                if (jt) {
                    int slot = 0;
                    if (lane == 0) slot = atomicAdd(&s_cnt3[(r + 1) % 3], jt);
                    slot = nbase + __shfl(slot, 0);
#pragma unroll
                    for (int q = 0; q < PEEL_UNROLL; q++) {
                        if (join[q]) s_Fq[slot + __popcll(jm[q] & below)] = (unsigned short)w[q];
                        slot += __popcll(jm[q]);
                    }
                }
            }
        }
        __syncthreads();
        left -= nF;
        fbase = nbase;
        nF = s_cnt3[(r + 1) % 3];
        r++;
        // the new frontier's decrements are over: its halves take its
        // sub-round (no barrier needed: see the level change above)
        for (int j = threadIdx.x; j < nF; j += blockDim.x) s_h16[s_Fq[fbase + j]] = (unsigned short)(r - r0);
        if (r > n) break;  // each sub-round removes a vertex: never reached
    }
    __syncthreads();
    // keys of every vertex of U
    for (int i = threadIdx.x; i < nu; i += blockDim.x) sub[uverts[i]] = r0 + (int)s_h16[i];
    if (threadIdx.x == 0) {
        ctl->subrounds = r;
        ctl->alpha = alpha;
        ctl->t_mark[3] = __builtin_amdgcn_s_memrealtime();
    }
}

// ------------------------------------------------- oriented CSR (N+(v))

__device__ __forceinline__ bool key_less(int su, int u, int sv, int v) {
    return su < sv || (su == sv && u < v);
}

// Rows of at most ORIENT_LANE_ROW entries are walked one vertex per lane
// (most rows of a sparse graph are short), longer ones by the whole wave.
#define ORIENT_LANE_ROW 32
// row entries a lane reads per step of such a row (loads in flight together)
#define ORIENT_UNROLL 8

// out-degree of every vertex; N+(v) (row order kept, so increasing id) is
// also written to tmp at v's own row start rp[v]: serial per lane, ballot
// compaction per wave.  Rows longer than PV_ORIENT_BLOCK_ROW are only
// listed in wlist[1..] (count in wlist[0]) for odeg_rows_kernel.
__global__ void __launch_bounds__(256) odeg_kernel(int n, const int *__restrict__ rp,
                                                    const int *__restrict__ col,
                                                    const int *__restrict__ sub,
                                                    int *__restrict__ odeg,
                                                    int *__restrict__ alpha, int *__restrict__ tmp,
                                                    int *__restrict__ wlist) {
    const int lane = threadIdx.x & 63;
    const int nw = (gridDim.x * blockDim.x) >> 6;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int amax = 0;
    for (int vb = ((blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64; vb < n; vb += nw * 64) {
        const int v = vb + lane;
        int b = 0, e = 0, sv = 0;
        if (v < n) {
            b = rp[v];
            e = rp[v + 1];
            sv = sub[v];
        }
        const bool huge = v < n && e - b > PV_ORIENT_BLOCK_ROW;
        const bool wide = v < n && e - b > ORIENT_LANE_ROW && !huge;
        int c = 0;
        if (huge) wlist[1 + atomicAdd(wlist, 1)] = v;
        if (v < n && !wide && !huge)
            // ORIENT_UNROLL entries a step: their column and key loads in
            // flight together rather than one dependent pair at a time
            for (int i0 = b; i0 < e; i0 += ORIENT_UNROLL) {
                int u[ORIENT_UNROLL], su[ORIENT_UNROLL];
#pragma unroll
                for (int q = 0; q < ORIENT_UNROLL; q++) u[q] = col[i0 + q < e ? i0 + q : i0];
#pragma unroll
                for (int q = 0; q < ORIENT_UNROLL; q++) su[q] = sub[u[q]];
#pragma unroll
                for (int q = 0; q < ORIENT_UNROLL; q++)
                    if (i0 + q < e && key_less(sv, v, su[q], u[q])) tmp[b + c++] = u[q];
            }
        for (uint64_t wm = ballot64(wide); wm; wm &= wm - 1ull) {
            const int L = __builtin_ctzll(wm);
            const int x = vb + L, sx = __shfl(sv, L, 64);
            const int xb = __shfl(b, L, 64), xe = __shfl(e, L, 64);
            int w = xb;
            for (int i0 = xb; i0 < xe; i0 += 64) {
                const int i = i0 + lane;
                bool take = false;
                int u = 0;
                if (i < xe) {
                    u = col[i];
                    take = key_less(sx, x, sub[u], u);
                }
                const uint64_t m = ballot64(take);
                if (take) tmp[w + __popcll(m & below)] = u;
                w += __popcll(m);
            }
            if (lane == L) c = w - xb;
        }
        if (v < n && !huge) odeg[v] = c;
        amax = max(amax, c);
    }
    amax = wave_max_i32(amax);
    if (lane == 0) atomicMax(alpha, amax);
}

// The listed long rows, a workgroup per row: each step a thread reads four
// consecutive entries, and a workgroup scan of the threads' take counts
// keeps N+(v) in row order
__global__ void __launch_bounds__(256) odeg_rows_kernel(const int *__restrict__ rp,
                                                         const int *__restrict__ col,
                                                         const int *__restrict__ sub,
                                                         int *__restrict__ odeg,
                                                         int *__restrict__ alpha, int *__restrict__ tmp,
                                                         const int *__restrict__ wide) {
    __shared__ int s_w[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nwide = wide[0];
    for (int t = blockIdx.x; t < nwide; t += gridDim.x) {
        const int x = wide[1 + t];
        const int sx = sub[x], xb = rp[x], xe = rp[x + 1];
        int w = xb;
        for (int i0 = xb; i0 < xe; i0 += 4 * 256) {
            const int base = i0 + 4 * (int)threadIdx.x;
            int u[4];
            bool tk[4];
#pragma unroll
            for (int q = 0; q < 4; q++) u[q] = (base + q < xe) ? col[base + q] : 0;
            int cnt = 0;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                tk[q] = base + q < xe && key_less(sx, x, sub[u[q]], u[q]);
                cnt += tk[q] ? 1 : 0;
            }
            const int inc = wave_incl_scan(cnt);
            if (lane == 63) s_w[wv] = inc;
            __syncthreads();
            int off = inc - cnt, tot = 0;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                off += (j < wv) ? s_w[j] : 0;
                tot += s_w[j];
            }
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (tk[q]) tmp[w + off++] = u[q];
            w += tot;
            __syncthreads();  // s_w is written again by the next step
        }
        if (threadIdx.x == 0) {
            odeg[x] = w - xb;
            atomicMax(alpha, w - xb);
        }
    }
}

// N+(v) moved from tmp (at rp[v]) to its place in the oriented CSR:
// contiguous copies, short rows per lane, long ones per wave
__global__ void __launch_bounds__(256) ofill_kernel(int n, const int *__restrict__ rp,
                                                     const int *__restrict__ tmp,
                                                     const int *__restrict__ orow,
                                                     int *__restrict__ ocol) {
    const int lane = threadIdx.x & 63;
    const int nw = (gridDim.x * blockDim.x) >> 6;
    for (int vb = ((blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64; vb < n; vb += nw * 64) {
        const int v = vb + lane;
        int b = 0, o = 0, d = 0;
        if (v < n) {
            b = rp[v];
            o = orow[v];
            d = orow[v + 1] - o;
        }
        const bool wide = d > ORIENT_LANE_ROW;
        if (!wide)
            for (int i = 0; i < d; i++) ocol[o + i] = tmp[b + i];
        for (uint64_t wm = ballot64(wide); wm; wm &= wm - 1ull) {
            const int L = __builtin_ctzll(wm);
            const int xb = __shfl(b, L, 64), xo = __shfl(o, L, 64), xd = __shfl(d, L, 64);
            for (int i = lane; i < xd; i += 64) ocol[xo + i] = tmp[xb + i];
        }
    }
}

// ---------------------------------------------------- exclusive scan (int)
// out[i] = sum_{j<i} in[j] for i <= n (out has n+1 entries).

#define SCAN_BLOCK 1024

__global__ void __launch_bounds__(256) scan_reduce_kernel(int n, const int *__restrict__ in,
                                                           int *__restrict__ bsum) {
    __shared__ int red[4];
    const int base = blockIdx.x * SCAN_BLOCK;
    int s = 0;
    for (int i = threadIdx.x; i < SCAN_BLOCK; i += 256)
        if (base + i < n) s += in[base + i];
    s = (int)wave_add_u32((uint32_t)s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(1024) scan_blocks_kernel(int nb, int *__restrict__ bsum) {
    // exclusive scan of nb block sums in place, one block of 1024 threads
    __shared__ int wsum[16];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += 1024) {
        const int i = base + threadIdx.x;
        const int x = (i < nb) ? bsum[i] : 0;
        const int inc = wave_incl_scan(x);
        if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = inc;
        __syncthreads();
        int off = carry;
        for (int w = 0; w < (int)(threadIdx.x >> 6); w++) off += wsum[w];
        if (i < nb) bsum[i] = off + inc - x;
        __syncthreads();
        if (threadIdx.x == 1023) carry = off + inc;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(1024) scan_apply_kernel(int n, const int *__restrict__ in,
                                                           const int *__restrict__ bsum,
                                                           int *__restrict__ out) {
    __shared__ int wsum[16];
    const int i = blockIdx.x * SCAN_BLOCK + threadIdx.x;
    const int x = (i < n) ? in[i] : 0;
    const int inc = wave_incl_scan(x);
    if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = inc;
    __syncthreads();
    int off = bsum[blockIdx.x];
    for (int w = 0; w < (int)(threadIdx.x >> 6); w++) off += wsum[w];
    if (i < n) out[i] = off + inc - x;
    if (i == n - 1) out[n] = off + inc;
}



// ------------------------------------------------------------- batches
// A batch of graphs is counted as their disjoint union: part b's vertices
// are renumbered voff_b + i and its columns shifted alike (a workgroup per
// part).  vgraph[v] names the part of union vertex v.
__global__ void __launch_bounds__(256) concat_kernel(const BatchPart *__restrict__ parts, int G,
                                                      int *__restrict__ rp, int *__restrict__ col,
                                                      int *__restrict__ vgraph) {
    for (int b = blockIdx.x; b < G; b += gridDim.x) {
        const BatchPart pt = parts[b];
        for (int i = threadIdx.x; i < pt.n; i += blockDim.x) {
            rp[pt.voff + i] = pt.rp[i] + (int)pt.eoff;
            vgraph[pt.voff + i] = b;
        }
        for (long long e = threadIdx.x; e < pt.nnz; e += blockDim.x) col[pt.eoff + e] = pt.col[e] + pt.voff;
    }
}

// ------------------------------------------------------------ edge ids
// The id of edge {u, v}, u < v, is its rank in lexicographic order: the
// position of v among the neighbours above u, after all such entries of
// rows 0..u-1.  ucnt[v] = number of neighbours above v, up = its
// exclusive scan; o2e maps each oriented CSR position to its edge id.

__global__ void __launch_bounds__(256) ucnt_kernel(int n, const int *__restrict__ rp,
                                                    const int *__restrict__ col,
                                                    int *__restrict__ ucnt) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        int lo = rp[v], hi = rp[v + 1];
        const int end = hi;
        while (lo < hi) {  // first neighbour > v
            const int mid = (lo + hi) >> 1;
            if (col[mid] <= v) lo = mid + 1;
            else hi = mid;
        }
        ucnt[v] = end - lo;
    }
}

__global__ void __launch_bounds__(256) o2e_kernel(int n, const int *__restrict__ rp,
                                                   const int *__restrict__ col,
                                                   const int *__restrict__ sub,
                                                   const int *__restrict__ orow,
                                                   const int *__restrict__ up,
                                                   int *__restrict__ o2e) {
    const int lane = threadIdx.x & 63;
    const int nw = (gridDim.x * blockDim.x) >> 6;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int v = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; v < n; v += nw) {
        const int sv = sub[v];
        const int r0 = rp[v], e1 = rp[v + 1];
        const int firstup = e1 - (up[v + 1] - up[v]);  // position of the first neighbour > v
        int w = orow[v];
        for (int e0 = r0; e0 < e1; e0 += 64) {
            const int e = e0 + lane;
            bool take = false;
            int u = 0;
            if (e < e1) {
                u = col[e];
                take = key_less(sv, v, sub[u], u);
            }
            const uint64_t m = ballot64(take);
            if (take) {
                int id;
                if (v < u) {
                    id = up[v] + (e - firstup);
                } else {
                    // v sits above u in u's row
                    int lo = rp[u], hi = rp[u + 1];
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (col[mid] < v) lo = mid + 1;
                        else hi = mid;
                    }
                    const int ufirst = rp[u + 1] - (up[u + 1] - up[u]);
                    // -1 only for an asymmetric CSR loaded unchecked
                    id = (lo < rp[u + 1] && col[lo] == v) ? up[u] + (lo - ufirst) : -1;
                }
                o2e[w + __popcll(m & below)] = id;
            }
            w += __popcll(m);
        }
    }
}

// ------------------------------------------------------- root buckets
// Counting sort of the roots by out-degree, largest first, so that heavy
// subtrees start early.  cnt has amax+2 slots.

// Three kernels without contended global atomics: every workgroup
// histograms a contiguous chunk of vertices in LDS, one workgroup turns the
// per-chunk histograms into output offsets (degree buckets largest first,
// chunks in order inside a bucket), and every workgroup scatters its chunk
// with LDS cursors.  bh is [chunks][PV_MAX_ALPHA + 1].
#define ROOT_BINS (PV_MAX_ALPHA + 1)

__global__ void __launch_bounds__(1024) root_hist_kernel(int n, int chunk, const int *__restrict__ amax_p,
                                                         const int *__restrict__ odeg,
                                                         int *__restrict__ bh) {
    __shared__ int h[ROOT_BINS];
    const int amax = *amax_p;
    if (amax > PV_MAX_ALPHA) return;  // refused by the host (PV_ETOOBIG)
    for (int d = threadIdx.x; d <= amax; d += blockDim.x) h[d] = 0;
    __syncthreads();
    const int v0 = blockIdx.x * chunk, v1 = min(n, v0 + chunk);
    for (int v = v0 + threadIdx.x; v < v1; v += blockDim.x) atomicAdd(&h[odeg[v]], 1);
    __syncthreads();
    for (int d = threadIdx.x; d <= amax; d += blockDim.x) bh[(long long)blockIdx.x * ROOT_BINS + d] = h[d];
}

// bh[b][d] becomes the first output slot of chunk b's roots of out-degree d
__global__ void __launch_bounds__(1024) root_offsets_kernel(int chunks, const int *__restrict__ amax_p,
                                                            int *__restrict__ bh, int *__restrict__ bounds,
                                                            int light_max) {
    __shared__ int tot[ROOT_BINS];
    __shared__ int start[ROOT_BINS];
    const int amax = *amax_p;
    if (amax > PV_MAX_ALPHA) return;  // refused by the host (PV_ETOOBIG)
    for (int d = threadIdx.x; d <= amax; d += blockDim.x) {
        int t = 0;
        for (int b = 0; b < chunks; b++) t += bh[(long long)b * ROOT_BINS + d];
        tot[d] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // buckets from the largest out-degree down
        int acc = 0;
        for (int d = amax; d >= 0; d--) {
            start[d] = acc;
            acc += tot[d];
        }
        // bounds[0] = #roots with d > light_max (heavy), bounds[1] = #roots with d >= 1
        bounds[0] = (light_max < amax) ? start[light_max] : 0;
        bounds[1] = start[0];
    }
    __syncthreads();
    for (int d = threadIdx.x; d <= amax; d += blockDim.x) {
        int acc = start[d];
        for (int b = 0; b < chunks; b++) {
            const int c = bh[(long long)b * ROOT_BINS + d];
            bh[(long long)b * ROOT_BINS + d] = acc;
            acc += c;
        }
    }
}

__global__ void __launch_bounds__(1024) root_scatter_kernel(int n, int chunk, const int *__restrict__ amax_p,
                                                            const int *__restrict__ odeg,
                                                            const int *__restrict__ bh,
                                                            int *__restrict__ order) {
    __shared__ int cur[ROOT_BINS];
    const int amax = *amax_p;
    if (amax > PV_MAX_ALPHA) return;  // refused by the host (PV_ETOOBIG)
    for (int d = threadIdx.x; d <= amax; d += blockDim.x) cur[d] = bh[(long long)blockIdx.x * ROOT_BINS + d];
    __syncthreads();
    const int v0 = blockIdx.x * chunk, v1 = min(n, v0 + chunk);
    for (int v = v0 + threadIdx.x; v < v1; v += blockDim.x) order[atomicAdd(&cur[odeg[v]], 1)] = v;
}

// ============================================================ host side

static int grid_for(long long items, int per_block, int cap) {
    long long b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

hipError_t pv_launch_check_rowptr(int n, long long nnz, const int *rp, int *d_err, hipStream_t s) {
    check_rowptr_kernel<<<grid_for((long long)n + 1, 256, 1 << 20), 256, 0, s>>>(n, nnz, rp, d_err);
    return hipGetLastError();
}

// only after the row pointers passed pv_launch_check_rowptr
hipError_t pv_launch_validate(int n, long long nnz, const int *rp, const int *col, int *d_err, hipStream_t s) {
    if (n <= 0 || nnz <= 0) return hipSuccess;
    // four waves per block, one chunk per wave and pass
    validate_kernel<<<grid_for((nnz + VALIDATE_CHUNK - 1) / VALIDATE_CHUNK, 4, 8192), 256, 0, s>>>(
        n, (int)nnz, rp, col, d_err);
    return hipGetLastError();
}

hipError_t pv_launch_peel(const DevInfo &dev, const PeelArgs &pa, hipStream_t s) {
    // co-resident blocks on a quarter of the CUs (8 per XCD on MI355X): a
    // grid barrier costs about 12 us with a block on every CU and under 5 us
    // with 64, and the sub-rounds' work does not need the wider grid (on a
    // 1M-vertex power-law graph the whole peel takes 15 ms instead of 21);
    // a single block when the graph already fits the solo phase
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, peel_kernel, PV_PEEL_THREADS, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const int blocks =
        (pa.n <= PV_SOLO_MAX) ? 1 : std::max(1, std::min(dev.num_cu / 4, PV_PEEL_MAX_BLOCKS));
    // An ordinary launch, not the cooperative API: the grid (at most a
    // quarter of the CUs, one block per CU as the occupancy query above
    // allows) is resident at once on the device, and the grid barrier's
    // wait is bounded, so a block that is not scheduled turns into an error
    // flag, not a hang.  Cooperative dispatches left the process to crash in
    // its exit handlers under the profiler, and an ordinary launch can also
    // be recorded into a HIP graph.
    if (blocks > per_cu * dev.num_cu) return hipErrorInvalidConfiguration;
    peel_kernel<<<blocks, PV_PEEL_THREADS, 0, s>>>(pa);
    return hipGetLastError();
}

hipError_t pv_launch_excl_scan(int n, const int *in, int *tmp, int *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    scan_reduce_kernel<<<nb, 256, 0, s>>>(n, in, tmp);
    scan_blocks_kernel<<<1, 1024, 0, s>>>(nb, tmp);
    scan_apply_kernel<<<nb, 1024, 0, s>>>(n, in, tmp, out);
    return hipGetLastError();
}

hipError_t pv_launch_orient(const DevInfo &dev, int n, const int *rp, const int *col, const int *sub,
                            int *odeg, int *orow, int *ocol, int *alpha, int *scan_tmp, int *row_tmp,
                            int *wide, hipStream_t s) {
    // a wave takes 64 vertices per step
    const int wblocks = grid_for((long long)n, 256, dev.num_cu * 32);
    hipError_t e = hipMemsetAsync(wide, 0, sizeof(int), s);
    if (e != hipSuccess) return e;
    odeg_kernel<<<wblocks, 256, 0, s>>>(n, rp, col, sub, odeg, alpha, row_tmp, wide);
    // the long rows, however many were listed: blocks without one exit
    odeg_rows_kernel<<<dev.num_cu * 2, 256, 0, s>>>(rp, col, sub, odeg, alpha, row_tmp, wide);
    (void)pv_launch_excl_scan(n, odeg, scan_tmp, orow, s);
    ofill_kernel<<<wblocks, 256, 0, s>>>(n, rp, row_tmp, orow, ocol);
    return hipGetLastError();
}

hipError_t pv_launch_root_order(int n, const int *amax, const int *odeg, int *bh, int chunks,
                                int *order, int *bounds, int light_max, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int chunk = (n + chunks - 1) / chunks;
    root_hist_kernel<<<chunks, 1024, 0, s>>>(n, chunk, amax, odeg, bh);
    root_offsets_kernel<<<1, 1024, 0, s>>>(chunks, amax, bh, bounds, light_max);
    root_scatter_kernel<<<chunks, 1024, 0, s>>>(n, chunk, amax, odeg, bh, order);
    return hipGetLastError();
}

hipError_t pv_launch_edge_ids(const DevInfo &dev, int n, const int *rp, const int *col, const int *sub,
                              const int *orow, int *ucnt, int *up, int *o2e, int *scan_tmp,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    ucnt_kernel<<<grid_for(n, 256, dev.num_cu * 32), 256, 0, s>>>(n, rp, col, ucnt);
    const int nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    scan_reduce_kernel<<<nb, 256, 0, s>>>(n, ucnt, scan_tmp);
    scan_blocks_kernel<<<1, 1024, 0, s>>>(nb, scan_tmp);
    scan_apply_kernel<<<nb, 1024, 0, s>>>(n, ucnt, scan_tmp, up);
    const int wblocks = grid_for((long long)n * 64, 256, dev.num_cu * 32);
    o2e_kernel<<<wblocks, 256, 0, s>>>(n, rp, col, sub, orow, up, o2e);
    return hipGetLastError();
}

hipError_t pv_launch_concat(const BatchPart *parts, int G, int maxn, int *rp, int *col, int *vgraph,
                            hipStream_t s) {
    (void)maxn;
    if (G <= 0) return hipSuccess;
    concat_kernel<<<std::min(G, 65535), 256, 0, s>>>(parts, G, rp, col, vgraph);
    return hipGetLastError();
}

// Out-degree histogram in powers of two (the graph part of a tuning key):
// per-block counts in LDS, one atomic per nonzero bucket and block.
__global__ void __launch_bounds__(256) deg_hist_kernel(int n, const int *__restrict__ odeg, int *__restrict__ hist) {
    __shared__ int s_h[PV_DEG_BUCKETS];
    if (threadIdx.x < PV_DEG_BUCKETS) s_h[threadIdx.x] = 0;
    __syncthreads();
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (long long)gridDim.x * blockDim.x) {
        const unsigned d = (unsigned)odeg[v];
        const int b = d ? min(32 - __builtin_clz(d), PV_DEG_BUCKETS - 1) : 0;
        atomicAdd(&s_h[b], 1);
    }
    __syncthreads();
    if (threadIdx.x < PV_DEG_BUCKETS && s_h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], s_h[threadIdx.x]);
}

hipError_t pv_launch_deg_hist(int n, const int *odeg, int *hist, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    deg_hist_kernel<<<grid_for(n, 256, 1024), 256, 0, s>>>(n, odeg, hist);
    return hipGetLastError();
}
