// Frequency distributions of local counts (Sec. 6, demonstrations: f_k(b),
// the number of vertices that take part in exactly b k-cliques).  From one
// column of a [rows][K] u128 table of local counts already in device
// memory: gather the column, sort it (bitonic network over a power-of-two
// padding, 128-bit keys compared high limb first), flag the first row of
// every run of equal values, scan the flags, and scatter each run's value
// and first position; a run's multiplicity is the gap to the next run.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "common.h"
#include "internal.h"

namespace {

__device__ __forceinline__ bool key_gt(uint64_t al, uint64_t ah, uint64_t bl, uint64_t bh) {
    return ah > bh || (ah == bh && al > bl);
}

// keys[i] = column `col` of row i; rows past the table sort last (all ones)
__global__ void __launch_bounds__(256) freq_gather_kernel(const uint64_t *__restrict__ src, long long rows, int K,
                                                          int col, long long npad, uint64_t *__restrict__ keys) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < npad;
         i += (long long)gridDim.x * blockDim.x) {
        uint64_t lo = ~0ull, hi = ~0ull;
        if (i < rows) {
            lo = src[2 * (i * K + col)];
            hi = src[2 * (i * K + col) + 1];
        }
        keys[2 * i] = lo;
        keys[2 * i + 1] = hi;
    }
}

// one compare-exchange step (block size k, partner distance j) of the
// bitonic network: element i and i ^ j, ascending where (i & k) == 0
__global__ void __launch_bounds__(256) bitonic_step_kernel(uint64_t *__restrict__ keys, long long npad, long long j,
                                                           long long k) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < npad;
         i += (long long)gridDim.x * blockDim.x) {
        const long long l = i ^ j;
        if (l <= i) continue;
        const uint64_t al = keys[2 * i], ah = keys[2 * i + 1];
        const uint64_t bl = keys[2 * l], bh = keys[2 * l + 1];
        const bool up = (i & k) == 0;
        if (up ? key_gt(al, ah, bl, bh) : key_gt(bl, bh, al, ah)) {
            keys[2 * i] = bl;
            keys[2 * i + 1] = bh;
            keys[2 * l] = al;
            keys[2 * l + 1] = ah;
        }
    }
}

// flags[i] = 1 where sorted row i starts a run of equal values
__global__ void __launch_bounds__(256) freq_flags_kernel(const uint64_t *__restrict__ keys, int rows,
                                                         int *__restrict__ flags) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += gridDim.x * blockDim.x)
        flags[i] = (i == 0 || keys[2 * i] != keys[2 * i - 2] || keys[2 * i + 1] != keys[2 * i - 1]) ? 1 : 0;
}

// run d (d = scanned flag) gets its value and first position
__global__ void __launch_bounds__(256) freq_scatter_kernel(const uint64_t *__restrict__ keys,
                                                           const int *__restrict__ flags,
                                                           const int *__restrict__ idx, int rows,
                                                           uint64_t *__restrict__ vals, int *__restrict__ pos) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += gridDim.x * blockDim.x) {
        if (!flags[i]) continue;
        const int d = idx[i];
        vals[2 * d] = keys[2 * i];
        vals[2 * d + 1] = keys[2 * i + 1];
        pos[d] = i;
    }
}

int grid_of(long long n) {
    const long long b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

// multiplicities: freq[d] = (next run's first position, or rows) - pos[d]
// for d < D = idx[rows]
__global__ void __launch_bounds__(256) freq_count_kernel(const int *__restrict__ idx, const int *__restrict__ pos,
                                                         int rows, uint64_t *__restrict__ freq) {
    const int D = idx[rows];
    for (int d = blockIdx.x * blockDim.x + threadIdx.x; d < D; d += gridDim.x * blockDim.x)
        freq[d] = (uint64_t)((d + 1 < D ? pos[d + 1] : rows) - pos[d]);
}

constexpr long long FS_ROWS = PV_FREQ_STATIC_ROWS;
constexpr long long FS_INTS = 3 * (FS_ROWS + 1) + FS_ROWS / 1024 + 2;
constexpr long long FS_WORDS = 2 * FS_ROWS + 2 * FS_ROWS + FS_ROWS + (FS_INTS + 1) / 2;
constexpr int FS_MAX_DEVICES = 64;

}  // namespace

// ------------------------------------------------ allocation-free variant
// One scratch array per device for pv_local_frequency_static (about 52 MiB,
// held by each device the library runs on until the process ends), in
// words: sort keys [2 npad], values [2 rows], multiplicities [rows], then
// int arrays flags, idx, pos [rows + 1 each] and the scan's block sums
// [rows / 1024 + 2]; npad <= rows <= PV_FREQ_STATIC_ROWS (a power of two).
// Every word a call reads is written earlier in the same call, so nothing
// has to start at zero; calls that overlap on one device race on it.
static __device__ __align__(256) uint64_t scratch[FS_WORDS];

// Its device address per device (in host code the name `scratch` is a
// host-side stand-in, not a device address), resolved once per device with
// that device current.
static uint64_t *g_scratch[FS_MAX_DEVICES];

// Called by pv_init with `device` current; resolves the address once per
// device (later contexts on the device find it set).
hipError_t pv_freq_static_init(int device) {
    if (device < 0 || device >= FS_MAX_DEVICES) return hipErrorInvalidDevice;
    if (__atomic_load_n(&g_scratch[device], __ATOMIC_ACQUIRE)) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    // two first contexts racing store the same address
    __atomic_store_n(&g_scratch[device], (uint64_t *)ptr, __ATOMIC_RELEASE);
    return hipSuccess;
}

hipError_t pv_launch_frequency_static(int device, const uint64_t *src, int rows, int K, int col, long long npad,
                                      uint64_t **vals, uint64_t **freq, int **idx, hipStream_t s) {
    if (device < 0 || device >= FS_MAX_DEVICES) return hipErrorInvalidDevice;
    uint64_t *base = __atomic_load_n(&g_scratch[device], __ATOMIC_ACQUIRE);
    if (!base) return hipErrorNotInitialized;
    if (rows > FS_ROWS || npad > FS_ROWS) return hipErrorInvalidValue;
    FreqWork w;
    w.keys = base;
    w.vals = base + 2 * FS_ROWS;
    uint64_t *fq = base + 4 * FS_ROWS;
    int *ints = (int *)(base + 5 * FS_ROWS);
    w.flags = ints;
    w.idx = ints + (FS_ROWS + 1);
    w.pos = ints + 2 * (FS_ROWS + 1);
    w.scan_tmp = ints + 3 * (FS_ROWS + 1);
    const hipError_t e = pv_launch_frequency(src, rows, K, col, npad, w, s);
    if (e != hipSuccess) return e;
    if (rows > 0) freq_count_kernel<<<grid_of(rows), 256, 0, s>>>(w.idx, w.pos, rows, fq);
    *vals = w.vals;
    *freq = fq;
    *idx = w.idx;
    return hipGetLastError();
}

hipError_t pv_launch_frequency(const uint64_t *src, int rows, int K, int col, long long npad, const FreqWork &w,
                               hipStream_t s) {
    freq_gather_kernel<<<grid_of(npad), 256, 0, s>>>(src, rows, K, col, npad, w.keys);
    for (long long k = 2; k <= npad; k <<= 1)
        for (long long j = k >> 1; j > 0; j >>= 1) bitonic_step_kernel<<<grid_of(npad), 256, 0, s>>>(w.keys, npad, j, k);
    if (rows <= 0) return hipGetLastError();
    freq_flags_kernel<<<grid_of(rows), 256, 0, s>>>(w.keys, rows, w.flags);
    hipError_t e = pv_launch_excl_scan(rows, w.flags, w.scan_tmp, w.idx, s);
    if (e != hipSuccess) return e;
    freq_scatter_kernel<<<grid_of(rows), 256, 0, s>>>(w.keys, w.flags, w.idx, rows, w.vals, w.pos);
    return hipGetLastError();
}
