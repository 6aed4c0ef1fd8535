// Fills and a device-wide exclusive scan (reduce-then-scan, three launches,
// fixed summation order so results are deterministic).
#include "internal.h"

namespace bake {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;  // 2048 values per block

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void fill_u8_kernel(uint8_t* p, uint8_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// Inclusive scan of one value per thread across a block of kScanBlock threads
// (wave64 shuffles, then the wave totals through LDS).  Returns the inclusive
// prefix; *block_total receives the block sum.
__device__ uint32_t block_inclusive_scan(uint32_t x, uint32_t* lds_waves, uint32_t* block_total) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds_waves[wave] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kScanBlock / 64; ++w) {
        uint32_t v = lds_waves[w];
        if (w < wave) base += v;
        tot += v;
    }
    __syncthreads();
    *block_total = tot;
    return x + base;
}

__global__ __launch_bounds__(kScanBlock) void scan_reduce_kernel(const uint32_t* in, int64_t n,
                                                                 uint32_t* block_sums) {
    __shared__ uint32_t lw[kScanBlock / 64];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)k * kScanBlock + threadIdx.x;
        if (i < n) acc += in[i];
    }
    uint32_t tot;
    block_inclusive_scan(acc, lw, &tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// Single block: exclusive scan of the block sums in place, total to *total.
__global__ __launch_bounds__(kScanBlock) void scan_sums_kernel(uint32_t* sums, int64_t nb,
                                                               uint32_t* total) {
    __shared__ uint32_t lw[kScanBlock / 64];
    uint32_t carry = 0;
    for (int64_t base = 0; base < nb; base += kScanBlock) {
        int64_t i = base + threadIdx.x;
        uint32_t v = i < nb ? sums[i] : 0;
        uint32_t tot;
        uint32_t inc = block_inclusive_scan(v, lw, &tot);
        if (i < nb) sums[i] = carry + inc - v;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

// Each block rescans its tile: thread t owns kScanItems consecutive values.
__global__ __launch_bounds__(kScanBlock) void scan_down_kernel(const uint32_t* in, uint32_t* out,
                                                               int64_t n,
                                                               const uint32_t* block_offs) {
    __shared__ uint32_t lw[kScanBlock / 64];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = i < n ? in[i] : 0;
        acc += v[k];
    }
    uint32_t tot;
    uint32_t inc = block_inclusive_scan(acc, lw, &tot);
    uint32_t run = block_offs[blockIdx.x] + inc - acc;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

// Single workgroup of 1024 threads for small arrays: tiles of 8192 values,
// each thread owning 8 consecutive ones, scanned through wave shuffles and
// LDS, with a running carry between tiles.
constexpr int kSmallBlock = 1024;
constexpr int kSmallItems = 8;
__global__ __launch_bounds__(kSmallBlock) void scan_small_kernel(const uint32_t* in, uint32_t* out,
                                                                 int64_t n, uint32_t* total) {
    __shared__ uint32_t lw[kSmallBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int64_t tile = 0; tile < n; tile += (int64_t)kSmallBlock * kSmallItems) {
        const int64_t b = tile + (int64_t)threadIdx.x * kSmallItems;
        uint32_t v[kSmallItems];
        uint32_t acc = 0;
#pragma unroll
        for (int k = 0; k < kSmallItems; ++k) {
            v[k] = b + k < n ? in[b + k] : 0u;
            acc += v[k];
        }
        uint32_t x = acc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) lw[wave] = x;
        __syncthreads();
        uint32_t base = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kSmallBlock / 64; ++w) {
            uint32_t t = lw[w];
            if (w < wave) base += t;
            tot += t;
        }
        __syncthreads();
        uint32_t run = carry + base + x - acc;
#pragma unroll
        for (int k = 0; k < kSmallItems; ++k) {
            if (b + k < n) out[b + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

int grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

}  // namespace

hipError_t fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u8_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp,
                              uint32_t* total, hipStream_t s) {
    if (n <= 0) {
        if (total) return fill_u32(total, 0, 1, s);
        return hipSuccess;
    }
    if (n <= (int64_t)kSmallBlock * kSmallItems * 16) {
        hipLaunchKernelGGL(scan_small_kernel, dim3(1), dim3(kSmallBlock), 0, s, in, out, n, total);
        return hipGetLastError();
    }
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n, tmp);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanBlock), 0, s, tmp, nb, total);
    hipLaunchKernelGGL(scan_down_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, out, n,
                       (const uint32_t*)tmp);
    return hipGetLastError();
}

}  // namespace bake
