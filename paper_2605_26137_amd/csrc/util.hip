// Fills, a device-wide exclusive scan (reduce-then-scan, three launches,
// fixed summation order so results are deterministic), the asset-table
// writer and the per-asset prefix tables that depend on device counts.
#include <string.h>

#include <algorithm>

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

// Table writer: one chunk of host bytes travels as a by-value kernel
// argument and is stored with vector writes.
constexpr int kChunkWords = 504;
struct TableChunk {
    uint32_t words;
    uint32_t pad;
    uint32_t w[kChunkWords];
};
__global__ __launch_bounds__(256) void table_chunk_kernel(uint32_t* dst, TableChunk c) {
    for (uint32_t i = threadIdx.x; i < c.words; i += 256) dst[i] = c.w[i];
}

// The first chunk, and zeroes of a region beside it (one launch for both):
// word set_idx of the region takes set_val instead.
__global__ __launch_bounds__(256) void table_zero_kernel(uint32_t* dst, TableChunk c, uint32_t* z, int64_t zwords,
                                                         int64_t set_idx, uint32_t set_val) {
    if (blockIdx.x == 0)
        for (uint32_t i = threadIdx.x; i < c.words; i += 256) dst[i] = c.w[i];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < zwords; i += (int64_t)gridDim.x * 256)
        z[i] = i == set_idx ? set_val : 0u;
}

// Exclusive prefix over the assets of a per-asset value, by one workgroup of
// 1024 threads in chunks of 1024 assets; out[n] receives the total.
constexpr int kPrefixBlock = 1024;
__device__ void asset_prefix(uint32_t v, int a, int n, uint32_t* out, uint32_t* carry_lds,
                             uint32_t* lw) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lw[wave] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int w = 0; w < kPrefixBlock / 64; ++w) {
        uint32_t t = lw[w];
        if (w < wave) base += t;
        tot += t;
    }
    const uint32_t carry = *carry_lds;
    if (a < n) out[a] = carry + base + x - v;
    __syncthreads();
    if (threadIdx.x == 0) *carry_lds = carry + tot;
    __syncthreads();
}

// After the raster: the ray list is the concatenation of the assets' face-
// ordered lists, and the exclusive scan of the per-face counts (total at
// index t_lf) gives every face's first ray.
// Also the prefix of the backward sort's tiles that will hold pairs (three
// per ray, kSortTile per tile) and their total beside the seal: the backward
// sort's grid covers every asset's capacity, and its blocks past the total
// exit on that one word.
__global__ __launch_bounds__(kPrefixBlock) void ray_spaces_kernel(Batch B, const uint32_t* face_off,
                                                                 int64_t t_lf, uint32_t* ray_pf,
                                                                 uint32_t* rb_pf, uint32_t* bt_pf) {
    __shared__ uint32_t lw[kPrefixBlock / 64];
    __shared__ uint32_t carry, carry_t;
    if (threadIdx.x == 0) carry = carry_t = 0;
    __syncthreads();
    for (int c = 0; c < B.n; c += kPrefixBlock) {
        const int a = c + threadIdx.x;
        uint32_t nb = 0, nt = 0;
        if (a < B.n) {
            const AssetDev& A = B.A[a];
            const uint32_t start = face_off[A.lf], end = face_off[A.lf + A.nlf];
            ray_pf[a] = start;
            B.cnt[(int64_t)a * kCntSlots + kCntRays] = end - start;
            nb = (end - start + 63u) / 64u;
            nt = (uint32_t)((3 * (uint64_t)(end - start) + kSortTile - 1) / kSortTile);
        }
        asset_prefix(nb, a, B.n, rb_pf, &carry, lw);
        asset_prefix(nt, a, B.n, bt_pf, &carry_t, lw);
    }
    if (threadIdx.x == 0) {
        ray_pf[B.n] = face_off[t_lf];
        rb_pf[B.n] = carry;
        bt_pf[B.n] = carry_t;
        B.gcnt[kGcBwdTiles] = carry_t;
    }
}

__global__ __launch_bounds__(kPrefixBlock) void treelet_space_kernel(Batch B, uint32_t* tl_pf) {
    __shared__ uint32_t lw[kPrefixBlock / 64];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int c = 0; c < B.n; c += kPrefixBlock) {
        const int a = c + threadIdx.x;
        uint32_t m = 0;
        if (a < B.n) {
            const uint32_t cap = (uint32_t)treelet_cap(B.A[a].nhf);
            m = min(B.cnt[(int64_t)a * kCntSlots + kCntTreelets], cap);
            if (B.A[a].nhf <= 1) m = 0;  // nothing to refit
        }
        asset_prefix(m, a, B.n, tl_pf, &carry, lw);
    }
    if (threadIdx.x == 0) tl_pf[B.n] = carry;
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
    if (n <= (int64_t)kSmallBlock * kSmallItems) {  // one tile: a single launch beats three
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

hipError_t write_table(void* dst, const void* src, size_t bytes, hipStream_t s, uint32_t* zero, int64_t zero_words,
                       int64_t set_idx, uint32_t set_val) {
    const uint32_t* w = (const uint32_t*)src;
    const size_t words = (bytes + 3) / 4;  // callers pass 4-byte multiples
    for (size_t o = 0; o < words || (o == 0 && zero_words > 0); o += kChunkWords) {
        TableChunk c;
        c.words = (uint32_t)std::min<size_t>(kChunkWords, words - std::min(o, words));
        c.pad = 0;
        memcpy(c.w, w + o, 4 * (size_t)c.words);
        if (o == 0 && zero_words > 0) {
            const unsigned g = (unsigned)std::min<int64_t>((zero_words + 255) / 256, 1024);
            hipLaunchKernelGGL(table_zero_kernel, dim3(g), dim3(256), 0, s, (uint32_t*)dst, c, zero, zero_words, set_idx,
                               set_val);
        } else {
            hipLaunchKernelGGL(table_chunk_kernel, dim3(1), dim3(256), 0, s, (uint32_t*)dst + o, c);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_ray_spaces(const BatchHost& H, hipStream_t s) {
    const Layout& L = H.L;
    hipLaunchKernelGGL(ray_spaces_kernel, dim3(1), dim3(kPrefixBlock), 0, s, H.dev,
                       (const uint32_t*)(H.ws + L.face_off), L.t_lf, (uint32_t*)(H.ws + L.ray_pf),
                       (uint32_t*)(H.ws + L.rb_pf), (uint32_t*)(H.ws + L.bt_pf));
    return hipGetLastError();
}

hipError_t launch_treelet_space(const BatchHost& H, hipStream_t s) {
    hipLaunchKernelGGL(treelet_space_kernel, dim3(1), dim3(kPrefixBlock), 0, s, H.dev,
                       (uint32_t*)(H.ws + H.L.tl_pf));
    return hipGetLastError();
}

}  // namespace bake
