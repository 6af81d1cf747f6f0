// Measured peaks of the device for the walk's roofline model: HBM stream
// copy and stream read, LDS 64-bit reads, and VALU integer lane operations
// of the pivot search's kind (XOR and popcount).  Each kernel does a known
// amount of work; the host times it with events and keeps the best rate.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "internal.h"

namespace {

__global__ void __launch_bounds__(256) peak_copy_kernel(const uint4 *__restrict__ a, uint4 *__restrict__ b,
                                                        long long n) {
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        b[i] = a[i];
}

__global__ void __launch_bounds__(256) peak_read_kernel(const uint4 *__restrict__ a, long long n,
                                                        unsigned *__restrict__ out) {
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const uint4 v = a[i];
        acc.x ^= v.x;
        acc.y ^= v.y;
        acc.z ^= v.z;
        acc.w ^= v.w;
    }
    out[blockIdx.x * 256 + threadIdx.x] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

// every lane reads consecutive 64-bit words (no bank conflicts): fifteen
// reads per iteration at immediate offsets from one address.  `zero` is 0;
// the compiler cannot know it, so the reads stay inside the loop.
__global__ void __launch_bounds__(256) peak_lds_kernel(int iters, int zero, unsigned long long *__restrict__ out) {
    __shared__ unsigned long long buf[4096];
    for (int i = threadIdx.x; i < 4096; i += 256) buf[i] = (unsigned long long)i * 0x9E3779B97F4A7C15ull;
    __syncthreads();
    unsigned long long a[4] = {0ull, 0ull, 0ull, 0ull};
    for (int it = 0; it < iters; it++) {
        const int base = (int)threadIdx.x + ((it * zero) & 255);  // <= 510: base + 256 * 14 < 4096
#pragma unroll
        for (int j = 0; j < PV_PEAK_LDS_READS; j++) a[j & 3] ^= buf[base + 256 * j];
    }
    out[blockIdx.x * 256 + threadIdx.x] = a[0] ^ a[1] ^ a[2] ^ a[3];
}

// eight independent chains of (XOR, popcount-accumulate): two VALU
// instructions per step
__global__ void __launch_bounds__(256) peak_valu_kernel(int iters, unsigned seed, unsigned *__restrict__ out) {
    unsigned a[8];
#pragma unroll
    for (int j = 0; j < 8; j++) a[j] = (threadIdx.x * 0x9E3779B9u) ^ (seed + 0x7F4A7C15u * (unsigned)j);
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int r = 0; r < 8; r++) {
#pragma unroll
            for (int j = 0; j < 8; j++) a[j] = __popc(a[j] ^ (seed + (unsigned)r)) + a[(j + 1) & 7];
        }
    }
    unsigned x = 0;
#pragma unroll
    for (int j = 0; j < 8; j++) x ^= a[j];
    out[blockIdx.x * 256 + threadIdx.x] = x;
}

}  // namespace

hipError_t pv_launch_peak_copy(const void *src, void *dst, long long bytes, hipStream_t s) {
    const long long n = bytes / 16;
    peak_copy_kernel<<<PV_PEAK_BLOCKS, 256, 0, s>>>((const uint4 *)src, (uint4 *)dst, n);
    return hipGetLastError();
}

hipError_t pv_launch_peak_read(const void *src, long long bytes, unsigned *sink, hipStream_t s) {
    const long long n = bytes / 16;
    peak_read_kernel<<<PV_PEAK_BLOCKS, 256, 0, s>>>((const uint4 *)src, n, sink);
    return hipGetLastError();
}

hipError_t pv_launch_peak_lds(int iters, int zero, unsigned long long *sink, hipStream_t s) {
    peak_lds_kernel<<<PV_PEAK_BLOCKS, 256, 0, s>>>(iters, zero, sink);
    return hipGetLastError();
}

hipError_t pv_launch_peak_valu(int iters, unsigned seed, unsigned *sink, hipStream_t s) {
    peak_valu_kernel<<<PV_PEAK_BLOCKS, 256, 0, s>>>(iters, seed, sink);
    return hipGetLastError();
}
