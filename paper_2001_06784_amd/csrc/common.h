// Internal helpers shared by the HIP translation units of libpivoter.
// CDNA (gfx950) only: 64-lane wavefronts, DPP cross-lane moves, scalar
// readlane/writelane for wave-uniform values.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define PV_WAVE 64

// ---------------------------------------------------------------- lanes

__device__ __forceinline__ int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint64_t ballot64(bool p) {
    return __builtin_amdgcn_ballot_w64(p);
}

// value of x in lane `l` (l wave-uniform) as a scalar
__device__ __forceinline__ uint32_t readlane32(uint32_t x, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int l) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// This lane's index computed afresh where it is used: a lane index the
// compiler hoists out of a walk's loop is one more register live across
// it, and under pressure it spills and comes back by a scratch load per
// use.  (volatile: neither hoisted nor merged; two VALU instructions)
__device__ __forceinline__ int lane_id_here() {
#if defined(__HIP_DEVICE_COMPILE__)
    int l;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
    return l;
#else
    return lane_id();
#endif
}

// x with lane `l` replaced by the wave-uniform value v (a compare and a
// select per 32-bit half)
__device__ __forceinline__ uint32_t writelane32(uint32_t x, uint32_t v, int l) {
    return (lane_id_here() == l) ? v : x;
}

__device__ __forceinline__ uint64_t writelane64(uint64_t x, uint64_t v, int l) {
    return (lane_id_here() == l) ? v : x;
}

// A value every lane holds alike, moved to scalar registers.  Values that
// arrive through vector loads stay in VGPRs otherwise, and then every
// bookkeeping step and branch on them costs vector instructions and exec
// masking.
__device__ __forceinline__ uint32_t uniform32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

__device__ __forceinline__ int uniformi(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// ------------------------------------------------- wave reductions (DPP)
// Full-wave max of an unsigned 32-bit value, returned wave-uniform.  Every
// lane of the wave must be active.  Quad swaps, half-row and row mirrors
// reduce each 16-lane row; row_bcast15/31 fold the four rows into lane 63.

// Lanes of rows outside ROWMASK read 0, the identity of unsigned max, so
// max(x, dpp(x)) leaves them unchanged; with that `old` value the compiler
// folds the move into the max (v_max_u32 with a DPP source).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWMASK, 0xF, false);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
    x = max(x, dpp_mov<0xB1, 0xF>(x));   // quad_perm [1,0,3,2]
    x = max(x, dpp_mov<0x4E, 0xF>(x));   // quad_perm [2,3,0,1]
    x = max(x, dpp_mov<0x141, 0xF>(x));  // row_half_mirror
    x = max(x, dpp_mov<0x140, 0xF>(x));  // row_mirror
    x = max(x, dpp_mov<0x142, 0xA>(x));  // row_bcast15 -> rows 1,3
    x = max(x, dpp_mov<0x143, 0xC>(x));  // row_bcast31 -> rows 2,3
    return readlane32(x, 63);
}

// Full-wave sum, returned wave-uniform, by the same DPP steps as
// wave_max_u32 (each step adds a disjoint partial sum; lanes outside a
// row mask read 0, the identity).  Every lane of the wave must be active.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
    x += dpp_mov<0xB1, 0xF>(x);   // quad pairs
    x += dpp_mov<0x4E, 0xF>(x);   // quads
    x += dpp_mov<0x141, 0xF>(x);  // half rows (the other quad)
    x += dpp_mov<0x140, 0xF>(x);  // rows (the other half)
    x += dpp_mov<0x142, 0xA>(x);  // rows 1, 3 add rows 0, 2
    x += dpp_mov<0x143, 0xC>(x);  // rows 2, 3 add rows 0 + 1
    return readlane32(x, 63);
}

// Full-wave bitwise OR, returned wave-uniform (the steps of wave_max_u32:
// OR is idempotent too).  Every lane of the wave must be active.
__device__ __forceinline__ uint32_t wave_or_u32(uint32_t x) {
    x |= dpp_mov<0xB1, 0xF>(x);
    x |= dpp_mov<0x4E, 0xF>(x);
    x |= dpp_mov<0x141, 0xF>(x);
    x |= dpp_mov<0x140, 0xF>(x);
    x |= dpp_mov<0x142, 0xA>(x);
    x |= dpp_mov<0x143, 0xC>(x);
    return readlane32(x, 63);
}

// Sum over the wave via cross-lane shuffles (not on the hot path).
__device__ __forceinline__ uint32_t wave_add_u32(uint32_t x) {
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ int wave_min_i32(int x) {
    for (int off = 32; off >= 1; off >>= 1) x = min(x, __shfl_xor(x, off, 64));
    return x;
}

__device__ __forceinline__ int wave_max_i32(int x) {
    for (int off = 32; off >= 1; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
    return x;
}

// inclusive prefix sum over the wave (lane order)
__device__ __forceinline__ int wave_incl_scan(int x) {
    const int lane = lane_id();
    for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// ------------------------------------------------------ exact 128-bit add
// out += (lo, hi) with two 64-bit device atomics; the carry out of the low
// limb is detected by the add that wraps it, so concurrent adds stay exact.
// Returns true if the high limb wrapped (the sum reached 2^128).
__device__ __forceinline__ bool atomic_add_u128(uint64_t *out, uint64_t lo, uint64_t hi) {
    bool ovf = false;
    if (lo) {
        uint64_t old = atomicAdd((unsigned long long *)out, (unsigned long long)lo);
        if (old + lo < old) {
            hi += 1;
            if (hi == 0) ovf = true;
        }
    }
    if (hi) {
        uint64_t old = atomicAdd((unsigned long long *)(out + 1), (unsigned long long)hi);
        if (old + hi < old) ovf = true;
    }
    return ovf;
}

// The same add in two halves, so that several can be in flight: first the
// low limb (returns the limb's old value), later the carry and high limb.
__device__ __forceinline__ uint64_t atomic_add_u128_lo(uint64_t *out, uint64_t lo) {
    return lo ? (uint64_t)atomicAdd((unsigned long long *)out, (unsigned long long)lo) : 0ull;
}

__device__ __forceinline__ bool atomic_add_u128_hi(uint64_t *out, uint64_t lo, uint64_t old, uint64_t hi) {
    bool ovf = false;
    if (lo && old + lo < old) {
        hi += 1;
        if (hi == 0) ovf = true;
    }
    if (hi) {
        const uint64_t o = atomicAdd((unsigned long long *)(out + 1), (unsigned long long)hi);
        if (o + hi < o) ovf = true;
    }
    return ovf;
}

// Make this wave's LDS / memory writes visible to its other lanes and keep
// the compiler from moving accesses across the point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int bcast0(int x) {
    return __builtin_amdgcn_readfirstlane(x);
}
