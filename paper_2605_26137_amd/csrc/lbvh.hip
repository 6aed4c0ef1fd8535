// LBVH build over the high-poly triangles (the paper's "GPU BVH built on the
// high-poly mesh", Sec. 6.4), after Karras 2012 (binary radix tree over sorted
// Morton codes):
//   1. reduction of the triangle-centroid bounds,
//   2. 30-bit Morton code of each centroid, value = original triangle index,
//   3. stable LSD radix sort of (code, index), 8-bit digits, LDS-ranked with
//      wave64 ballots, so equal codes keep ascending index order,
//   4. Karras hierarchy: every internal node finds its key range and split
//      from common-prefix lengths (code, extended by the index on equal codes);
//      the same kernel packs the leaves (vertices copied bit-exactly, original
//      index kept) and lists the refit's treelets and the nodes above them,
//   5. bottom-up refit in LDS, treelet by treelet, then the nodes above the
//      treelets: the second arriving child of a node unions both boxes and
//      continues upward (min/max is exact, so the boxes do not depend on
//      arrival order); the nodes are then written compressed (32 B each).
// In a batch every asset gets its own tree over its own bounds; sort tiles
// never straddle two assets, and each tile places its keys from its asset's
// per-tile and per-super-tile digit counts (section 3).
#include <algorithm>
#include <utility>

#include "internal.h"

namespace bake {

namespace {

constexpr int kBlock = 256;
constexpr int kSortBlock = 1024;                     // sort workgroups: 16 waves
constexpr int kSortRounds = kSortTile / kSortBlock;  // 4 keys per thread and pass
constexpr int kSortWaves = kSortBlock / 64;
constexpr float kLeafEps = 1.0f / 16384.0f;  // edge tolerance of the hit rule (traverse.hip)

__device__ __forceinline__ int3 tri_idx(const int32_t* __restrict__ F, int64_t g, int64_t nv,
                                        bool* bad) {
    int32_t a = F[3 * g], b = F[3 * g + 1], c = F[3 * g + 2];
    bool ok = a >= 0 && b >= 0 && c >= 0 && a < nv && b < nv && c < nv;
    *bad = !ok;
    if (!ok) a = b = c = 0;  // degenerate stand-in: never hit, never out of bounds
    return make_int3(a, b, c);
}

__device__ __forceinline__ float3 ldv(const float* __restrict__ V, int32_t i) {
    return make_float3(V[3 * (int64_t)i], V[3 * (int64_t)i + 1], V[3 * (int64_t)i + 2]);
}

__device__ __forceinline__ float3 centroid(const float* __restrict__ V, int3 t) {
    float3 a = ldv(V, t.x), b = ldv(V, t.y), c = ldv(V, t.z);
    const float k = 1.0f / 3.0f;
    return make_float3((a.x + b.x + c.x) * k, (a.y + b.y + c.y) * k, (a.z + b.z + c.z) * k);
}

__device__ __forceinline__ int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// 1. centroid bounds: a partial per sort tile, then one workgroup per asset
// ---------------------------------------------------------------------------

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ void block_minmax6(float v[6], float* out) {
    __shared__ float red[kBlock / 64][6];
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = wave_min(v[k]);
#pragma unroll
    for (int k = 3; k < 6; ++k) v[k] = wave_max(v[k]);
    if (lane == 0)
        for (int k = 0; k < 6; ++k) red[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            for (int k = 0; k < 3; ++k) v[k] = fminf(v[k], red[w][k]);
            for (int k = 3; k < 6; ++k) v[k] = fmaxf(v[k], red[w][k]);
        }
        for (int k = 0; k < 6; ++k) out[k] = v[k];
    }
}

__global__ __launch_bounds__(kBlock) void bounds_part_kernel(Batch Bt, float* __restrict__ part) {
    // kBoundsSplit workgroups per sort tile, each over its 1/kBoundsSplit of it
    int64_t lt;
    const int sub = (int)(blockIdx.x % kBoundsSplit);
    const AssetDev& As = Bt.A[block_asset(Bt, kGSort, blockIdx.x / kBoundsSplit, &lt)];
    const float* __restrict__ V = As.hi_V;
    const int32_t* __restrict__ F = As.hi_F;
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    bool anybad = false, nonfin = false;
    constexpr int64_t kPart = kSortTile / kBoundsSplit;
    const int64_t first = lt * kSortTile + sub * kPart;
    const int64_t end = min((int64_t)As.nhf, first + kPart);
    // kU triangles per thread and trip, their index and vertex loads issued
    // together (one gather latency per trip instead of per triangle)
    constexpr int kU = 4;
    for (int64_t g0 = first + threadIdx.x; g0 < end; g0 += kU * kBlock) {
        int3 t[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            bool bad = false;
            const int64_t g = g0 + (int64_t)u * kBlock;
            t[u] = g < end ? tri_idx(F, g, As.nhv, &bad) : make_int3(0, 0, 0);
            anybad |= bad;
        }
        float3 c[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) c[u] = centroid(V, t[u]);
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (g0 + (int64_t)u * kBlock >= end) continue;
            if (!(isfinite(c[u].x) && isfinite(c[u].y) && isfinite(c[u].z))) {
                nonfin = true;
                continue;
            }
            v[0] = fminf(v[0], c[u].x); v[1] = fminf(v[1], c[u].y); v[2] = fminf(v[2], c[u].z);
            v[3] = fmaxf(v[3], c[u].x); v[4] = fmaxf(v[4], c[u].y); v[5] = fmaxf(v[5], c[u].z);
        }
    }
    if (anybad) set_status(Bt, kStHiIndex);
    if (nonfin) set_status(Bt, kStNonFinite);
    block_minmax6(v, part + 6 * (kBoundsSplit * (As.stile + lt) + sub));
}

__global__ __launch_bounds__(kBlock) void bounds_final_kernel(Batch Bt, const float* __restrict__ part,
                                                              float* __restrict__ bounds) {
    const AssetDev& As = Bt.A[blockIdx.x];
    const int64_t nparts = kBoundsSplit * ceil_div(As.nhf, kSortTile);
    const float* p = part + 6 * kBoundsSplit * As.stile;
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = threadIdx.x; i < nparts; i += kBlock) {
        for (int k = 0; k < 3; ++k) v[k] = fminf(v[k], p[6 * i + k]);
        for (int k = 3; k < 6; ++k) v[k] = fmaxf(v[k], p[6 * i + k]);
    }
    block_minmax6(v, bounds + 6 * (int64_t)blockIdx.x);
}

// ---------------------------------------------------------------------------
// 2. Morton codes (value = asset-local triangle index)
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t spread10(uint32_t x) {
    // 10 bits -> every third bit of 30
    x &= 0x3FFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ __forceinline__ uint32_t quant10(float c, float lo, float inv) {
    float q = (c - lo) * inv * 1024.0f;
    q = fminf(fmaxf(q, 0.0f), 1023.0f);  // NaN -> 0
    return (uint32_t)q;
}

__global__ __launch_bounds__(kBlock) void morton_kernel(Batch Bt, const float* __restrict__ bounds_all,
                                                        uint32_t* __restrict__ keys,
                                                        uint32_t* __restrict__ vals) {
    int64_t lb;
    const int a = block_asset(Bt, kGHiF, blockIdx.x, &lb);
    const AssetDev& As = Bt.A[a];
    const int64_t g = lb * kBlock + threadIdx.x;
    if (g >= As.nhf) return;
    const float* bounds = bounds_all + 6 * (int64_t)a;
    bool bad;
    int3 t = tri_idx(As.hi_F, g, As.nhv, &bad);
    float3 c = centroid(As.hi_V, t);
    float ex = bounds[3] - bounds[0], ey = bounds[4] - bounds[1], ez = bounds[5] - bounds[2];
    float ix = ex > 0.f ? 1.0f / ex : 0.f, iy = ey > 0.f ? 1.0f / ey : 0.f,
          iz = ez > 0.f ? 1.0f / ez : 0.f;
    uint32_t x = quant10(c.x, bounds[0], ix), y = quant10(c.y, bounds[1], iy),
             z = quant10(c.z, bounds[2], iz);
    keys[As.hf + g] = (spread10(x) << 2) | (spread10(y) << 1) | spread10(z);
    vals[As.hf + g] = (uint32_t)g;
}

// ---------------------------------------------------------------------------
// 3. stable LSD radix sort, 8-bit digits, per asset
// ---------------------------------------------------------------------------

// Digit offsets without a separate scan.  A pass is two launches: the
// histogram kernel writes each tile's 256 digit counts as a row
// (hist[hbase + 256 lt + digit]) and adds them into its super-tile's row
// (kSuper consecutive tiles of one asset, sup[sbase + 256 (lt / kSuper) +
// digit], integer atomics: the sums do not depend on their order); the
// scatter kernel then finds where its tile's keys of digit d start from
//   start + (the asset's keys with a smaller digit: all super-tile rows)
//         + (earlier tiles' keys of digit d: earlier super-tiles' rows and the
//            rows of the earlier tiles in its own super-tile),
// which is the exclusive scan of the counts in (digit, tile) order.
// The tile of a sort block: its asset's keys [start, start + count) in the
// concatenated arrays, its count row (hbase + 256 lt), its super-tile rows
// (from sbase; an asset's super-tiles start at tile_base / kSuper + asset,
// which keeps assets apart) and its local tile lt.  BWD: the backward pairs,
// whose count lives on the device (three per ray), with tiles sized for the
// capacity 3 res^2.
struct SortTile {
    int64_t start, count, hbase, sbase, lt;
};

// BWD blocks map onto the tiles that hold pairs (the prefix the forward wrote
// after its raster); the grid covers the capacity, and its blocks past the
// pairs' tiles have exited already (bwd_block_idle).
template <bool BWD>
__device__ __forceinline__ SortTile sort_tile(const Batch& Bt, int64_t blk) {
    SortTile T;
    int a;
    if (BWD) {
        a = upper_asset(Bt.bt_pf, Bt.n, blk);
        T.lt = blk - Bt.bt_pf[a];
    } else {
        a = block_asset(Bt, kGSort, blk, &T.lt);
    }
    const AssetDev& As = Bt.A[a];
    const int64_t tile_base = BWD ? As.btile : As.stile;
    if (BWD) {
        T.start = 3 * (int64_t)Bt.ray_pf[a];
        T.count = 3 * (int64_t)Bt.cnt[(int64_t)a * kCntSlots + kCntRays];
    } else {
        T.start = As.hf;
        T.count = As.nhf;
    }
    T.hbase = 256 * tile_base;
    T.sbase = 256 * (tile_base / kSuper + a);
    return T;
}

// A backward sort block with nothing to do: a workspace no longer holding the
// saved forward, or a block past the tiles that hold pairs.  Both words lie
// in one line of the batch counters, so an idle block exits after one load
// latency.
__device__ __forceinline__ bool bwd_block_idle(const Batch& Bt) {
    return !sealed(Bt) || blockIdx.x >= Bt.gcnt[kGcBwdTiles];
}

template <bool BWD>
__global__ __launch_bounds__(kSortBlock) void radix_hist_kernel(Batch Bt, const uint32_t* __restrict__ keys,
                                                                int shift, uint32_t* __restrict__ hist,
                                                                uint32_t* __restrict__ sup) {
    __shared__ uint32_t h[256];
    if (BWD && bwd_block_idle(Bt)) return;
    const SortTile T = sort_tile<BWD>(Bt, blockIdx.x);
    if (T.lt * kSortTile >= T.count) return;  // an empty capacity tile (uniform)
    if (threadIdx.x < 256) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = T.lt * kSortTile;
    // all rounds' keys are loaded before the first count (one load latency)
    uint32_t k[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + (int64_t)r * kSortBlock + threadIdx.x;
        k[r] = i < T.count ? keys[T.start + i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r)
        if (base + (int64_t)r * kSortBlock + threadIdx.x < T.count) atomicAdd(&h[(k[r] >> shift) & 255u], 1u);
    __syncthreads();
    if (threadIdx.x < 256) {
        const uint32_t c = h[threadIdx.x];
        hist[T.hbase + 256 * T.lt + threadIdx.x] = c;
        if (c) atomicAdd(&sup[T.sbase + 256 * (T.lt / kSuper) + threadIdx.x], c);
    }
}

// Element r*1024 + tid of the block's tile is ranked among equal digits by
// (earlier rounds, earlier waves, earlier lanes): a stable order.  The tile is
// first placed in LDS in that order (digit runs contiguous), then written out
// with consecutive lanes on consecutive positions of each run.  The tile's
// first position of each digit comes from the count rows (see kSuper).  The
// keys are loaded first, so that their latency overlaps the reads of the
// count rows.  Ranking: each wave finds, per round, the lanes of each digit
// (ballots over the digit's bits) and records their count for its (round,
// wave, digit); one scan per digit over the 64 (round, wave) counts, in that
// order, then turns the counts into positions, so the whole tile is ranked
// between two barriers.
template <bool BWD>
__global__ __launch_bounds__(kSortBlock) void radix_scatter_kernel(Batch Bt, const uint32_t* __restrict__ kin,
                                                                   const uint32_t* __restrict__ vin,
                                                                   uint32_t* __restrict__ kout,
                                                                   uint32_t* __restrict__ vout, int shift,
                                                                   const uint32_t* __restrict__ hist,
                                                                   const uint32_t* __restrict__ sup) {
    __shared__ uint32_t s_key[kSortTile];  // also the scratch of the count-row sums
    __shared__ uint32_t s_val[kSortTile];
    __shared__ uint32_t s_loc[256];   // tile-local first position of each digit
    __shared__ uint32_t s_glob[256];  // global position of the tile's first key of each digit
    __shared__ uint32_t s_run[256];   // the tile's digit counts
    __shared__ uint32_t s_wsum[4];
    __shared__ uint32_t s_part[kSortRounds][256];  // per round: the digit's keys in the round
    // per (round, wave, digit): the count, then the tile-local first position
    __shared__ uint16_t wcnt[kSortRounds][kSortWaves][256];
    static_assert(kSortTile <= 65535, "tile positions are kept in 16 bits");
    static_assert(kSortBlock == 4 * 256 && kSortRounds * kSortWaves == 64, "one scan thread per (round, digit)");
    if (BWD && bwd_block_idle(Bt)) return;
    const SortTile T = sort_tile<BWD>(Bt, blockIdx.x);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = T.lt * kSortTile;
    const int64_t nvalid = min((int64_t)kSortTile, T.count - base);
    if (nvalid <= 0) return;  // an empty capacity tile (uniform)
    uint32_t key[kSortRounds], val[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = (int64_t)r * kSortBlock + tid;
        const bool valid = i < nvalid;
        key[r] = valid ? kin[T.start + base + i] : 0u;
        val[r] = valid ? vin[T.start + base + i] : 0u;
    }
    uint32_t(*scratch)[256] = reinterpret_cast<uint32_t(*)[256]>(s_key);
    {
        // per digit, in four parts: the asset's count (all super-tile rows)
        // and the count before this tile (earlier super-tiles, then the
        // earlier tiles of its own super-tile)
        // (the loads of a group are all issued before their sums: one load
        // latency per group instead of one per row)
        const int d = tid & 255, part = tid >> 8;
        const int64_t S = T.lt / kSuper, nS = ceil_div(ceil_div(T.count, kSortTile), kSuper);
        uint32_t tot = 0, before = 0;
        uint32_t hv[kSuper / 4];
#pragma unroll
        for (int j = 0; j < kSuper / 4; ++j) {
            const int64_t t = S * kSuper + part + 4 * j;
            hv[j] = t < T.lt ? hist[T.hbase + 256 * t + d] : 0u;
        }
        for (int64_t x0 = part; x0 < nS; x0 += 4 * 8) {
            uint32_t v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int64_t x = x0 + 4 * j;
                v[j] = x < nS ? sup[T.sbase + 256 * x + d] : 0u;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                tot += v[j];
                if (x0 + 4 * j < S) before += v[j];
            }
        }
#pragma unroll
        for (int j = 0; j < kSuper / 4; ++j) before += hv[j];
        scratch[part][d] = tot;
        scratch[4 + part][d] = before;
    }
    __syncthreads();
    uint32_t tot = 0, before = 0;
    if (tid < 256) {
        tot = (scratch[0][tid] + scratch[1][tid]) + (scratch[2][tid] + scratch[3][tid]);
        before = (scratch[4][tid] + scratch[5][tid]) + (scratch[6][tid] + scratch[7][tid]);
        // exclusive scan of the asset's digit counts (waves 0-3)
        uint32_t x = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) s_wsum[wave] = x;
        tot = x - tot;  // exclusive within the wave
    }
    __syncthreads();
    if (tid < 256) {
        uint32_t w = 0;
        for (int k = 0; k < wave; ++k) w += s_wsum[k];
        s_glob[tid] = (uint32_t)T.start + w + tot + before;
        s_run[tid] = 0;
    }
    for (int x = tid; x < kSortRounds * kSortWaves * 256 / 2; x += kSortBlock)
        reinterpret_cast<uint32_t*>(&wcnt[0][0][0])[x] = 0;
    __syncthreads();
    // the tile's digit counts, and every wave's per-round digit counts
    uint32_t rank[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const bool valid = (int64_t)r * kSortBlock + tid < nvalid;
        const uint32_t dig = (key[r] >> shift) & 255u;
        if (valid) atomicAdd(&s_run[dig], 1u);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dig >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        rank[r] = (uint32_t)__popcll(peers & __lanemask_lt());
        if (valid && rank[r] == 0) wcnt[r][wave][dig] = (uint16_t)__popcll(peers);
    }
    __syncthreads();
    // thread (rr, d): exclusive scan of digit d's counts over the waves of
    // round rr; waves 0-3 also scan the tile's digit counts
    const int sd = tid & 255, rr = tid >> 8;
    uint32_t ex[kSortWaves];
    {
        uint32_t acc = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
            ex[w] = acc;
            acc += wcnt[rr][w][sd];
        }
        s_part[rr][sd] = acc;
    }
    uint32_t c = 0, x = 0;
    if (tid < 256) {
        c = s_run[tid];
        x = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) s_wsum[wave] = x;
    }
    __syncthreads();
    if (tid < 256) {
        uint32_t b = 0;
        for (int w = 0; w < wave; ++w) b += s_wsum[w];
        s_loc[tid] = b + x - c;
    }
    __syncthreads();
    {
        uint32_t p = s_loc[sd];
        for (int r = 0; r < rr; ++r) p += s_part[r][sd];
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) wcnt[rr][w][sd] = (uint16_t)(p + ex[w]);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        if ((int64_t)r * kSortBlock + tid < nvalid) {
            const uint32_t dig = (key[r] >> shift) & 255u;
            const uint32_t pos = (uint32_t)wcnt[r][wave][dig] + rank[r];
            s_key[pos] = key[r];
            s_val[pos] = val[r];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int e = r * kSortBlock + tid;
        if (e >= nvalid) break;
        const uint32_t k = s_key[e];
        const uint32_t d = (k >> shift) & 255u;
        const uint32_t pos = s_glob[d] + ((uint32_t)e - s_loc[d]);
        if ((int64_t)pos < T.start + T.count) {  // always, unless the counts were corrupted
            kout[pos] = k;
            vout[pos] = s_val[e];
        } else {
            set_status(Bt, kStInternal);
        }
    }
}

// ---------------------------------------------------------------------------
// 4. Karras hierarchy
// ---------------------------------------------------------------------------

// Per-thread search reach: a node's range and split are searched by its own
// thread in the wave's LDS window of sorted keys when the range spans at most
// kKarrasReach keys; longer ranges (the few nodes near the top) are searched
// by the whole wave together, 64 probes per step.
constexpr int kKarrasReach = 64;
// Leaves per refit treelet (section 5): the hierarchy kernel lists the treelets.
constexpr int kTreelet = 2048;

// The largest x in [lo, hi) with pred(x), given pred(lo) and not pred(hi)
// (pred monotone: true up to some point, false after it); the wave searches
// 64 candidates per step.  Wave-uniform arguments.
template <typename Pred>
__device__ __forceinline__ int64_t wave_last_true(int64_t lo, int64_t hi, int lane, Pred pred) {
    while (hi - lo > 1) {
        const int64_t step = (hi - lo + 63) / 64;
        const int64_t x = lo + (int64_t)lane * step;
        const bool ok = lane > 0 && x < hi && pred(x);
        const uint64_t m = __ballot(ok) | 1ull;
        const int last = 63 - __clzll((long long)m);
        lo += (int64_t)last * step;
        hi = min(hi, lo + step);
    }
    return lo;
}

// Appends, for every lane with want set, one slot of the per-asset list whose
// length counter is *counter: one atomic per wave (the wave's asset is
// uniform), slots in lane order.  Returns the lane's slot.
__device__ __forceinline__ uint32_t wave_append(uint32_t* counter, bool want) {
    const uint64_t m = __ballot(want);
    if (m == 0) return 0;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = __shfl(base, leader, 64);
    return base + (uint32_t)__popcll(m & __lanemask_lt());
}

// Also packs leaf i (its triangle's corners and index, in sorted order: the
// leaves are independent of the hierarchy) and lists the refit's work (see
// section 5): a node of more than kTreelet
// leaves is a top node, listed with its parent link (by its parent, or by
// itself at the root); a child of at most kTreelet leaves of a top node, or
// a root of at most kTreelet leaves, roots a treelet, listed with its range
// and parent link.  Clears the arrival counters of the refit's fallback.
__global__ __launch_bounds__(kBlock) void karras_kernel(Batch Bt, const uint32_t* __restrict__ keys_all,
                                                        const uint32_t* __restrict__ sorted_idx,
                                                        Leaf* __restrict__ leaves,
                                                        uint32_t* __restrict__ child_all,
                                                        int32_t* __restrict__ np_all,
                                                        int32_t* __restrict__ lp_all,
                                                        int4* __restrict__ list_all,
                                                        int2* __restrict__ top_all,
                                                        uint32_t* __restrict__ cnt_all) {
    // each wave's window: keys [i0 - 64, i0 + 128) around its nodes [i0, i0 + 64)
    __shared__ uint32_t s_win[kBlock / 64][3 * 64];
    int64_t lb;
    const int a = block_asset(Bt, kGHiF, blockIdx.x, &lb);
    const AssetDev& As = Bt.A[a];
    const int64_t n = As.nhf;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i0 = lb * kBlock + wave * 64;
    const int64_t i = i0 + lane;
    if (i < n) {
        const uint32_t g = sorted_idx[As.hf + i];
        bool bad;
        const int3 t = tri_idx(As.hi_F, g, As.nhv, &bad);
        const float3 va = ldv(As.hi_V, t.x), vb = ldv(As.hi_V, t.y), vc = ldv(As.hi_V, t.z);
        Leaf lf;
        lf.a = make_float4(va.x, va.y, va.z, vb.x);
        lf.b = make_float4(vb.y, vb.z, vc.x, vc.y);
        lf.c = make_float4(vc.z, __int_as_float((int32_t)g), 0.f, 0.f);
        leaves[As.hf + i] = lf;
    }
    const uint32_t* __restrict__ keys = keys_all + As.hf;
    uint32_t* win = s_win[wave];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int64_t q = i0 - 64 + 64 * r + lane;
        if (q >= 0 && q < n) win[64 * r + lane] = keys[q];
    }
    __syncthreads();
    if (i0 >= n - 1) return;  // the whole wave is past the asset's nodes
    // common-prefix length of keys a and b (b within the window of a's wave;
    // extended by the indices on equal keys), -1 outside [0, n)
    auto cpw = [&](int64_t a, int64_t b) -> int {
        if (b < 0 || b >= n) return -1;
        const uint32_t x = win[a - i0 + 64], y = win[b - i0 + 64];
        return x == y ? 32 + __clz((uint32_t)a ^ (uint32_t)b) : __clz(x ^ y);
    };
    const bool live = i < n - 1;
    int d = 1, dmin = 0, dnode = 0;
    int64_t l = 0, sp = 0;
    bool big = false;
    if (live) {
        d = (cpw(i, i + 1) - cpw(i, i - 1)) >= 0 ? 1 : -1;
        dmin = cpw(i, i - d);
        int64_t lmax = 2;
        while (lmax <= kKarrasReach && cpw(i, i + lmax * d) > dmin) lmax <<= 1;
        if (lmax > kKarrasReach) {
            big = true;
        } else {
            for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
                if (cpw(i, i + (l + t) * d) > dmin) l += t;
            dnode = cpw(i, i + l * d);
            int64_t t = l;
            do {
                t = (t + 1) >> 1;
                if (cpw(i, i + (sp + t) * d) > dnode) sp += t;
            } while (t > 1);
        }
    }
    // the wave's long ranges, one at a time: range end by probing the powers
    // of two, then 64-way refinement; the split likewise
    uint64_t bm = __ballot(big);
    while (bm) {
        const int src = __ffsll((long long)bm) - 1;
        bm &= bm - 1;
        const int64_t bi = __shfl(i, src, 64);
        const int bd = __shfl(d, src, 64), bdmin = __shfl(dmin, src, 64);
        const uint32_t kb = keys[bi];
        auto cpg = [&](int64_t b) -> int {
            if (b < 0 || b >= n) return -1;
            const uint32_t y = keys[b];
            return kb == y ? 32 + __clz((uint32_t)bi ^ (uint32_t)b) : __clz(kb ^ y);
        };
        // 2^k for k <= 6 is known to lie in the range (the per-thread search
        // found 64 in it); lanes 7..40 probe 2^lane
        const bool okp = lane > 6 && lane <= 40 && cpg(bi + ((int64_t)1 << lane) * bd) > bdmin;
        const uint64_t m = __ballot(okp) | 0x7Full;
        const int K = 63 - __clzll((long long)m);
        const int64_t L = wave_last_true((int64_t)1 << K, (int64_t)1 << (K + 1), lane,
                                         [&](int64_t x) { return cpg(bi + x * bd) > bdmin; });
        const int bdnode = cpg(bi + L * bd);
        const int64_t S = wave_last_true(0, L, lane, [&](int64_t x) { return cpg(bi + x * bd) > bdnode; });
        if (lane == src) {
            l = L;
            dnode = bdnode;
            sp = S;
        }
    }
    if (!live) return;
    int32_t* __restrict__ node_parent = np_all + As.node;
    int32_t* __restrict__ leaf_parent = lp_all + As.hf;
    const int64_t j = i + l * d;
    (void)dnode;
    const int64_t gamma = i + sp * d + (d < 0 ? -1 : 0);
    const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    const int32_t left = lo == gamma ? ~(int32_t)gamma : (int32_t)gamma;
    const int32_t right = hi == gamma + 1 ? ~(int32_t)(gamma + 1) : (int32_t)(gamma + 1);
    child_all[As.node + i] = (uint32_t)gamma | (left < 0 ? kChildLeafL : 0u) | (right < 0 ? kChildLeafR : 0u);
    if (left < 0) leaf_parent[gamma] = (int32_t)(i << 1);
    else node_parent[gamma] = (int32_t)(i << 1);
    if (right < 0) leaf_parent[gamma + 1] = (int32_t)((i << 1) | 1);
    else node_parent[gamma + 1] = (int32_t)((i << 1) | 1);
    if (i == 0) node_parent[0] = -1;
    // the refit's lists
    cnt_all[As.node + i] = 0u;
    const bool top = hi - lo + 1 > kTreelet;
    const uint32_t cap = (uint32_t)treelet_cap(n);
    uint32_t* ntop = &Bt.cnt[(int64_t)a * kCntSlots + kCntTop];
    uint32_t* ntl = &Bt.cnt[(int64_t)a * kCntSlots + kCntTreelets];
    const int32_t cref[2] = {left, right};
    const int32_t clo[2] = {(int32_t)lo, (int32_t)(gamma + 1)}, chi[2] = {(int32_t)gamma, (int32_t)hi};
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int32_t pp = (int32_t)((i << 1) | side);
        const bool cbig = chi[side] - clo[side] + 1 > kTreelet;
        const uint32_t et = wave_append(ntop, cbig);
        if (cbig) {
            if (et < cap) top_all[As.tl + et] = make_int2(cref[side], pp);
            else set_status(Bt, kStInternal);
        }
        const bool root = top && !cbig;
        const uint32_t e = wave_append(ntl, root);
        if (root) {
            if (e < cap) list_all[As.tl + e] = make_int4(cref[side], clo[side], chi[side], pp);
            else set_status(Bt, kStInternal);
        }
    }
    const uint32_t er = wave_append(top ? ntop : ntl, i == 0);
    if (i == 0) {
        if (er >= cap) set_status(Bt, kStInternal);
        else if (top) top_all[As.tl + er] = make_int2(0, -1);
        else list_all[As.tl + er] = make_int4(0, 0, (int32_t)(n - 1), -1);
    }
}

// ---------------------------------------------------------------------------
// 5. leaves + refit
// ---------------------------------------------------------------------------
//
// The refit avoids device-scope ordering per node (an acquire/release at
// device scope costs an L2 write-back and invalidation across the XCDs, and
// chains of them serialise the upper levels):
//  a. treelets: the maximal subtrees with at most kTreelet leaves (listed by
//     the hierarchy kernel).  A Karras node covers a contiguous leaf range
//     [lo, hi] and its index lies in that range, so a treelet's internal
//     nodes have indices in [lo, hi] too;
//  b. one workgroup per treelet loads the parent links of [lo, hi] into LDS
//     and refits bottom-up: each child leaves its box in its own LDS slot of
//     the parent (one slot per side) and counts its arrival in LDS; the second
//     arrival reads the sibling's slot and continues.  The treelet root's box
//     goes to its parent's slot and the parent is appended to a frontier; the
//     workgroup then writes the treelet's nodes compressed, in parallel;
//  c. one workgroup per asset finishes the nodes above the treelets from the
//     frontier: in LDS when there are at most kTopLds of them, else with
//     global counters that only this workgroup touches.

constexpr int kRefitBlock = 1024;  // 16 waves: the LDS footprint allows one workgroup per CU
constexpr int kTopBlock = 1024;
constexpr int kTopList = 8192;

__device__ __forceinline__ void put_slot(BvhNode* node, int side, const float b[6]) {
    float* f = reinterpret_cast<float*>(node) + 6 * side;
#pragma unroll
    for (int k = 0; k < 6; ++k) f[k] = b[k];
}

__device__ __forceinline__ float pow2f(uint32_t e) { return __uint_as_float(e << 23); }  // 2^(e - 127)

// One axis of a compressed node: the frame [o, o + 255 s] with s a power of
// two, and the bytes of the four child planes.  A decoded plane fmaf(v, s, o)
// rounds lo + v s once, and lo + v s is exact whenever it is representable,
// so it lies on the outer side of a plane c exactly when lo + v s does: the
// bytes come from (c - lo) / s (exact scaling of a once-rounded difference,
// off by at most one) and one check each.
__device__ __forceinline__ uint32_t quantise_axis(float lL, float hL, float lR, float hR, float* o_out,
                                                  uint32_t q_out[4]) {
    const float lo = fminf(lL, lR), hi = fmaxf(hL, hR);
    if (!(isfinite(lo) && isfinite(hi) && lo <= hi)) {
        // NaN planes: an unbounded slab in the box tests
        *o_out = __uint_as_float(0x7FC00000u);
        q_out[0] = q_out[1] = q_out[2] = q_out[3] = 0;
        return 127u;
    }
    // ext / 2^(E - 7) lies in [128, 256) for ext in [2^E, 2^(E+1)); one
    // doubling when 255 steps still fall short of hi
    const float ext = hi - lo;
    const uint32_t eb = (__float_as_uint(ext) >> 23) & 0xFFu;
    uint32_t e = eb > 8u ? eb - 7u : 1u;
    if (e < 254u && fmaf(255.f, pow2f(e), lo) < hi) ++e;
    const float s = pow2f(e), inv = pow2f(254u - e);  // inv = 1 / s
    const float pl[4] = {lL, hL, lR, hR};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float c = pl[j];
        const float x = fminf(fmaxf((c - lo) * inv, 0.f), 255.f);
        uint32_t v;
        if ((j & 1) == 0) {  // lower plane: the largest v with lo + v s <= c
            v = (uint32_t)floorf(x);
            if (v > 0u && fmaf((float)v, s, lo) > c) --v;
        } else {             // upper plane: the smallest v with lo + v s >= c
            v = (uint32_t)ceilf(x);
            if (v < 255u && fmaf((float)v, s, lo) < c) ++v;
        }
        q_out[j] = v;
    }
    *o_out = lo;
    return e;
}

// Writes node p whole: its frame, child planes and child word (the
// hierarchy kernel's), two 16-B stores.
__device__ __forceinline__ void write_compressed(BvhNodeC* node, uint32_t child, const float L[6], const float R[6]) {
    float o[3];
    uint32_t q[3][4], e[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) e[k] = quantise_axis(L[k], L[k + 3], R[k], R[k + 3], &o[k], q[k]);
    // byte order: L.lo.xyz, L.hi.xyz, R.lo.xyz, R.hi.xyz
    const uint32_t b[12] = {q[0][0], q[1][0], q[2][0], q[0][1], q[1][1], q[2][1],
                            q[0][2], q[1][2], q[2][2], q[0][3], q[1][3], q[2][3]};
    uint32_t w[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) w[i] = b[4 * i] | (b[4 * i + 1] << 8) | (b[4 * i + 2] << 16) | (b[4 * i + 3] << 24);
    node->a = make_float4(o[0], o[1], o[2], __uint_as_float(e[0] | (e[1] << 8) | (e[2] << 16)));
    node->q = make_uint4(w[0], w[1], w[2], child);
}


// Box of a leaf triangle, widened for the hit rule's edge tolerance: weights
// down to -kLeafEps put the crossing inside the triangle scaled by (1 + 3
// kLeafEps) about its centroid; widen by 4 kLeafEps of the extent (3 plus
// rounding margin) and a few ulps of the coordinates.
__device__ __forceinline__ void leaf_box(const Leaf& L, float box[6]) {
    float ax = L.a.x, ay = L.a.y, az = L.a.z, bx = L.a.w, by = L.b.x, bz = L.b.y;
    float cx = L.b.z, cy = L.b.w, cz = L.c.x;
    box[0] = fminf(fminf(ax, bx), cx); box[1] = fminf(fminf(ay, by), cy); box[2] = fminf(fminf(az, bz), cz);
    box[3] = fmaxf(fmaxf(ax, bx), cx); box[4] = fmaxf(fmaxf(ay, by), cy); box[5] = fmaxf(fmaxf(az, bz), cz);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        float ext = box[q + 3] - box[q];
        float pad = 4.0f * kLeafEps * ext + 4.76837158e-7f * fmaxf(fabsf(box[q]), fabsf(box[q + 3]));
        box[q] -= pad;
        box[q + 3] += pad;
    }
}

// Workgroups take the batch's treelets in turn (the treelet prefix over the
// assets is known on the device only).
__global__ __launch_bounds__(kRefitBlock) void treelet_refit_kernel(
    Batch Bt, const Leaf* __restrict__ leaves_all, BvhNode* nodes_all, BvhNodeC* __restrict__ nodes_c_all,
    const uint32_t* __restrict__ child_all,
    const int32_t* __restrict__ np_all,
    const int32_t* __restrict__ lp_all, const int4* __restrict__ list_all, int32_t* __restrict__ frontier_all) {
    __shared__ int32_t s_np[kTreelet];      // parent link of internal node lo + i
    __shared__ int32_t s_lp[kTreelet];      // parent link of leaf lo + i
    __shared__ uint32_t s_cnt[kTreelet];    // arrivals at internal node lo + i
    __shared__ float s_box[kTreelet][2][6]; // child boxes of internal node lo + i, by side
    const uint32_t total = Bt.tl_pf[Bt.n];
    for (uint32_t g = blockIdx.x; g < total; g += gridDim.x) {
        const int a = upper_asset(Bt.tl_pf, Bt.n, g);
        const AssetDev& As = Bt.A[a];
        const int64_t n = As.nhf;
        const Leaf* __restrict__ leaves = leaves_all + As.hf;
        BvhNode* nodes = nodes_all + As.node;
        BvhNodeC* __restrict__ nodes_c = nodes_c_all + As.node;
        const uint32_t* __restrict__ child = child_all + As.node;
        const int32_t* __restrict__ node_parent = np_all + As.node;
        const int32_t* __restrict__ leaf_parent = lp_all + As.hf;
        uint32_t* nfront = &Bt.cnt[(int64_t)a * kCntSlots + kCntFrontier];
        const uint32_t front_cap = (uint32_t)treelet_cap(n);
        const int4 T = list_all[As.tl + (g - Bt.tl_pf[a])];
        const int32_t ref = T.x, lo = T.y, hi = T.z, rootpp = T.w;
        const int32_t sz = hi - lo + 1;
        for (int i = threadIdx.x; i < sz; i += kRefitBlock) {
            s_np[i] = (lo + i < n - 1) ? node_parent[lo + i] : -1;
            s_lp[i] = n > 1 ? leaf_parent[lo + i] : -1;
            s_cnt[i] = 0;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < sz; i += kRefitBlock) {
            float box[6];
            leaf_box(leaves[lo + i], box);
            int32_t cur = ~(lo + i);   // node whose box is in `box`
            int32_t pp = s_lp[i];
            for (int level = 0;; ++level) {
                if (cur == ref) {
                    // treelet complete: hand its box to the node above
                    if (rootpp >= 0) {
                        put_slot(&nodes[rootpp >> 1], rootpp & 1, box);
                        uint32_t e = atomicAdd(nfront, 1u);
                        if (e < front_cap) frontier_all[As.tl + e] = rootpp;
                        else set_status(Bt, kStInternal);
                    }
                    break;
                }
                if (level > 2 * kMaxDepth || pp < 0) {  // only a malformed hierarchy gets here
                    set_status(Bt, kStInternal);
                    break;
                }
                const int32_t p = pp >> 1, side = pp & 1, li = p - lo;
                if (li < 0 || li >= sz) {  // only a malformed hierarchy gets here
                    set_status(Bt, kStInternal);
                    break;
                }
                // each child leaves its box in its own LDS slot of p and
                // counts its arrival; the second arrival (workgroup-scope
                // acquire) reads the other slot and writes the node out
#pragma unroll
                for (int q = 0; q < 6; ++q) s_box[li][side][q] = box[q];
                uint32_t old = __hip_atomic_fetch_add(&s_cnt[li], 1u, __ATOMIC_ACQ_REL,
                                                      __HIP_MEMORY_SCOPE_WORKGROUP);
                if (old == 0) break;
                float sib[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) sib[q] = s_box[li][1 - side][q];

#pragma unroll
                for (int q = 0; q < 3; ++q) box[q] = fminf(box[q], sib[q]);
#pragma unroll
                for (int q = 3; q < 6; ++q) box[q] = fmaxf(box[q], sib[q]);
                cur = p;
                pp = s_np[li];
            }
        }
        __syncthreads();
        // the treelet's internal nodes (both children arrived) from their LDS
        // slots, in parallel
        for (int i = threadIdx.x; i < sz; i += kRefitBlock)
            if (s_cnt[i] == 2u) write_compressed(&nodes_c[lo + i], child[lo + i], s_box[i][0], s_box[i][1]);
        __syncthreads();
    }
}

// Top pass: one workgroup per asset climbs from its frontier through the nodes
// above the treelets.  Each frontier entry says: child `side` of node p is
// complete and its box is in p's slot.
//
// When the asset has at most kTopLds top nodes, the climb runs in LDS: the
// top nodes (listed by karras_kernel) get LDS slots through an LDS
// hash of their indices, each learns its parent's slot, the frontier's boxes
// are copied into their parents' LDS box slots, and the climb's arrival
// counters, parent links and boxes are LDS accesses only.  Otherwise the
// nodes' global box slots and counters serve.
constexpr int kTopLds = 2048;
constexpr int kTopHash = 4096;  // open addressing, linear probing (load <= 1/2)

__device__ __forceinline__ uint32_t top_hash(int32_t p) { return ((uint32_t)p * 2654435761u) >> 20; }

__device__ __forceinline__ int top_slot(const int32_t* hkey, const int16_t* hval, int32_t p) {
    uint32_t h = top_hash(p) & (kTopHash - 1);
    for (int probe = 0; probe < kTopHash; ++probe) {
        const int32_t k = hkey[h];
        if (k == p) return hval[h];
        if (k == -1) return -1;
        h = (h + 1) & (kTopHash - 1);
    }
    return -1;
}

struct TopLds {
    int32_t hkey[kTopHash];
    int16_t hval[kTopHash];
    int32_t node[kTopLds];      // top node of slot e
    int32_t up[kTopLds];        // parent slot link (slot << 1 | side), -1 at the root
    uint32_t cnt[kTopLds];      // arrivals
    float box[kTopLds][2][6];   // child boxes, by side
};

__device__ void refit_top_lds(Batch Bt, const AssetDev& As, BvhNode* nodes, BvhNodeC* __restrict__ nodes_c,
                              const uint32_t* __restrict__ child, const int32_t* __restrict__ frontier, uint32_t nf,
                              const int2* __restrict__ top, uint32_t nt, TopLds& S) {
    int32_t* s_hkey = S.hkey;
    int16_t* s_hval = S.hval;
    int32_t* s_node = S.node;
    int32_t* s_up = S.up;
    uint32_t* s_cnt = S.cnt;
    float(*s_box)[2][6] = S.box;
    const int tid = threadIdx.x;
    for (int h = tid; h < kTopHash; h += kTopBlock) s_hkey[h] = -1;
    __syncthreads();
    for (uint32_t e = tid; e < nt; e += kTopBlock) {
        const int2 t = top[e];
        s_node[e] = t.x;
        s_cnt[e] = 0;
        uint32_t h = top_hash(t.x) & (kTopHash - 1);
        for (int probe = 0; probe < kTopHash; ++probe) {
            if (atomicCAS(&s_hkey[h], -1, t.x) == -1) {
                s_hval[h] = (int16_t)e;
                break;
            }
            h = (h + 1) & (kTopHash - 1);
        }
    }
    __syncthreads();
    for (uint32_t e = tid; e < nt; e += kTopBlock) {
        const int32_t pp = top[e].y;
        int32_t up = -1;
        if (pp >= 0) {
            const int ps = top_slot(s_hkey, s_hval, pp >> 1);
            if (ps < 0) set_status(Bt, kStInternal);  // a top node's parent is a top node
            else up = (ps << 1) | (pp & 1);
        }
        s_up[e] = up;
    }
    // the treelet roots' boxes, from their parents' global slots
    for (uint32_t f = tid; f < nf; f += kTopBlock) {
        const int32_t pp = frontier[f];
        const int ps = top_slot(s_hkey, s_hval, pp >> 1);
        if (ps < 0) {
            set_status(Bt, kStInternal);
            continue;
        }
        const float* g = reinterpret_cast<const float*>(&nodes[pp >> 1]) + 6 * (pp & 1);
#pragma unroll
        for (int q = 0; q < 6; ++q) s_box[ps][pp & 1][q] = g[q];
    }
    __syncthreads();
    for (uint32_t f = tid; f < nf; f += kTopBlock) {
        const int32_t pp0 = frontier[f];
        int e = top_slot(s_hkey, s_hval, pp0 >> 1);
        for (int level = 0; e >= 0; ++level) {
            if (level > 2 * kMaxDepth) {  // only a malformed hierarchy gets here
                set_status(Bt, kStInternal);
                break;
            }
            const uint32_t old = __hip_atomic_fetch_add(&s_cnt[e], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0) break;
            float box[6];
#pragma unroll
            for (int q = 0; q < 3; ++q) box[q] = fminf(s_box[e][0][q], s_box[e][1][q]);
#pragma unroll
            for (int q = 3; q < 6; ++q) box[q] = fmaxf(s_box[e][0][q], s_box[e][1][q]);
            const int32_t up = s_up[e];
            if (up < 0) break;
#pragma unroll
            for (int q = 0; q < 6; ++q) s_box[up >> 1][up & 1][q] = box[q];
            e = up >> 1;
        }
    }
    __syncthreads();
    for (uint32_t e = tid; e < nt; e += kTopBlock) {
        if (s_cnt[e] == 2u) write_compressed(&nodes_c[s_node[e]], child[s_node[e]], s_box[e][0], s_box[e][1]);
        else set_status(Bt, kStInternal);
    }
}

__global__ __launch_bounds__(kTopBlock) void refit_top_kernel(Batch Bt, BvhNode* nodes_all,
                                                             BvhNodeC* __restrict__ nodes_c_all,
                                                             const uint32_t* __restrict__ child_all,
                                                             const int32_t* __restrict__ np_all,
                                                             const int32_t* __restrict__ frontier_all,
                                                             const int2* __restrict__ top_all,
                                                             uint32_t* cnt_all) {
    // global path: nodes completed by the climb, compressed in parallel after
    // it (beyond the list's capacity a node is compressed where it completes)
    union TopMem {
        TopLds lds;
        int32_t done[kTopList];
    };
    __shared__ TopMem s_mem;
    __shared__ uint32_t s_ndone;
    int32_t* s_done = s_mem.done;
    const int a = blockIdx.x;
    const AssetDev& As = Bt.A[a];
    if (As.nhf <= 1) return;
    BvhNode* nodes = nodes_all + As.node;
    BvhNodeC* __restrict__ nodes_c = nodes_c_all + As.node;
    const uint32_t* __restrict__ child = child_all + As.node;
    const int32_t* __restrict__ node_parent = np_all + As.node;
    const int32_t* __restrict__ frontier = frontier_all + As.tl;
    uint32_t* cnt = cnt_all + As.node;
    const uint32_t m = min(Bt.cnt[(int64_t)a * kCntSlots + kCntFrontier], (uint32_t)treelet_cap(As.nhf));
    const uint32_t nt = Bt.cnt[(int64_t)a * kCntSlots + kCntTop];
    if (nt > 0 && nt <= min((uint32_t)kTopLds, (uint32_t)treelet_cap(As.nhf))) {
        refit_top_lds(Bt, As, nodes, nodes_c, child, frontier, m, top_all + As.tl, nt, s_mem.lds);
        return;
    }
    if (threadIdx.x == 0) s_ndone = 0;
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < m; e += kTopBlock) {
        int32_t pp = frontier[e];
        for (int level = 0; pp >= 0; ++level) {
            if (level > 2 * kMaxDepth) {
                set_status(Bt, kStInternal);
                break;
            }
            int32_t p = pp >> 1;
            uint32_t old = __hip_atomic_fetch_add(&cnt[p], 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0) break;
            float box[6], bl[6], br[6];
            const float* f = reinterpret_cast<const float*>(&nodes[p]);
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                bl[q] = f[q];
                br[q] = f[6 + q];
            }
            const uint32_t slot = atomicAdd(&s_ndone, 1u);
            if (slot < (uint32_t)kTopList) s_done[slot] = p;
            else write_compressed(&nodes_c[p], child[p], bl, br);
#pragma unroll
            for (int q = 0; q < 3; ++q) box[q] = fminf(bl[q], br[q]);
#pragma unroll
            for (int q = 3; q < 6; ++q) box[q] = fmaxf(bl[q], br[q]);
            pp = node_parent[p];
            if (pp >= 0) put_slot(&nodes[pp >> 1], pp & 1, box);
        }
    }
    __syncthreads();
    const uint32_t nd = min(s_ndone, (uint32_t)kTopList);
    for (uint32_t i = threadIdx.x; i < nd; i += kTopBlock) {
        const int32_t p = s_done[i];
        const float* f = reinterpret_cast<const float*>(&nodes[p]);
        float bl[6], br[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            bl[q] = f[q];
            br[q] = f[6 + q];
        }
        write_compressed(&nodes_c[p], child[p], bl, br);
    }
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

int64_t bwd_sort_zero_words(const Layout& L) {
    return L.save ? sort_super_rows(L.t_btile, L.n) * 256 * (int64_t)kSortPasses : 0;
}

hipError_t launch_sort(const BatchHost& H, int which, int bits, bool* result_in_1, hipStream_t s,
                       hipEvent_t after_first) {
    const Layout& L = H.L;
    const bool bwd = which == kSortBwd;
    const int64_t blocks = H.blocks(bwd ? kGBwdSort : kGSort);
    *result_in_1 = false;
    const int passes = (bits + 7) / 8;
    if (blocks == 0 || passes == 0) return after_first ? hipEventRecord(after_first, s) : hipSuccess;
    uint32_t* kin = (uint32_t*)(H.ws + (bwd ? L.bwd_k0 : L.keys0));
    uint32_t* vin = (uint32_t*)(H.ws + (bwd ? L.bwd_v0 : L.vals0));
    uint32_t* kout = (uint32_t*)(H.ws + (bwd ? L.bwd_k1 : L.keys1));
    uint32_t* vout = (uint32_t*)(H.ws + (bwd ? L.bwd_v1 : L.vals1));
    uint32_t* hist = (uint32_t*)(H.ws + (bwd ? L.bwd_hist : L.hist));
    uint32_t* sup = (uint32_t*)(H.ws + (bwd ? L.bwd_sup : L.sup));
    const int64_t sup_pass = sort_super_rows(bwd ? L.t_btile : L.t_stile, L.n) * 256;
    if (passes > kSortPasses) return hipErrorInvalidValue;
    // the super-tile rows start at zero: the BVH sort's lie in the region
    // every forward zeroes first, the backward's are zeroed with the
    // backward's gradient table (bwd_sort_zero_words)
    hipError_t e = hipSuccess;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        uint32_t* sp = sup + sup_pass * p;
        if (bwd) {
            hipLaunchKernelGGL(radix_hist_kernel<true>, dim3((unsigned)blocks), dim3(kSortBlock), 0, s, H.dev,
                               (const uint32_t*)kin, shift, hist, sp);
            if (p == 0 && after_first && (e = hipEventRecord(after_first, s)) != hipSuccess) return e;
            hipLaunchKernelGGL(radix_scatter_kernel<true>, dim3((unsigned)blocks), dim3(kSortBlock), 0, s, H.dev,
                               (const uint32_t*)kin, (const uint32_t*)vin, kout, vout, shift,
                               (const uint32_t*)hist, (const uint32_t*)sp);
        } else {
            hipLaunchKernelGGL(radix_hist_kernel<false>, dim3((unsigned)blocks), dim3(kSortBlock), 0, s, H.dev,
                               (const uint32_t*)kin, shift, hist, sp);
            if (p == 0 && after_first && (e = hipEventRecord(after_first, s)) != hipSuccess) return e;
            hipLaunchKernelGGL(radix_scatter_kernel<false>, dim3((unsigned)blocks), dim3(kSortBlock), 0, s, H.dev,
                               (const uint32_t*)kin, (const uint32_t*)vin, kout, vout, shift,
                               (const uint32_t*)hist, (const uint32_t*)sp);
        }
        std::swap(kin, kout);
        std::swap(vin, vout);
        *result_in_1 = !*result_in_1;
    }
    return hipGetLastError();
}

hipError_t launch_bvh_build(const BatchHost& H, hipStream_t s) {
    const Layout& L = H.L;
    if (L.t_hf <= 0) return hipSuccess;
    char* ws = H.ws;
    hipError_t e;
    float* part = (float*)(ws + L.bounds_part);
    float* bounds = (float*)(ws + L.bounds);
    uint32_t* k0 = (uint32_t*)(ws + L.keys0);
    uint32_t* v0 = (uint32_t*)(ws + L.vals0);
    BvhNode* nodes = (BvhNode*)(ws + L.nodes);
    BvhNodeC* nodes_c = (BvhNodeC*)(ws + L.nodes_c);
    Leaf* leaves = (Leaf*)(ws + L.leaves);
    int32_t* np = (int32_t*)(ws + L.node_parent);
    int32_t* lp = (int32_t*)(ws + L.leaf_parent);
    uint32_t* cnt = (uint32_t*)(ws + L.refit_cnt);
    int32_t* frontier = (int32_t*)(ws + L.frontier);
    int4* tlist = (int4*)(ws + L.treelets);
    int2* top = (int2*)(ws + L.top);
    uint32_t* child = (uint32_t*)(ws + L.child);

    hipLaunchKernelGGL(bounds_part_kernel, dim3((unsigned)(H.blocks(kGSort) * kBoundsSplit)), dim3(kBlock), 0, s,
                       H.dev, part);
    hipLaunchKernelGGL(bounds_final_kernel, dim3((unsigned)L.n), dim3(kBlock), 0, s, H.dev,
                       (const float*)part, bounds);
    hipLaunchKernelGGL(morton_kernel, dim3((unsigned)H.blocks(kGHiF)), dim3(kBlock), 0, s, H.dev,
                       (const float*)bounds, k0, v0);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    bool in1 = false;
    if ((e = launch_sort(H, kSortBvh, 30, &in1, s)) != hipSuccess) return e;
    // 30-bit keys take four 8-bit passes: the sorted arrays are back in keys0 / vals0
    if (H.blocks(kGHiF) > 0) {
        hipLaunchKernelGGL(karras_kernel, dim3((unsigned)H.blocks(kGHiF)), dim3(kBlock), 0, s, H.dev,
                           (const uint32_t*)k0, (const uint32_t*)v0, leaves, child, np, lp, tlist, top, cnt);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (L.t_node > 0) {
        if ((e = launch_treelet_space(H, s)) != hipSuccess) return e;
        // enough workgroups for the treelets of every asset (at least one per
        // kTreelet / 2 leaves), capped
        int64_t grid = 0;
        for (int a = 0; a < L.n; ++a) grid += H.A[a].nhf / (kTreelet / 2) + 1;
        grid = std::min<int64_t>(grid, 2048);
        hipLaunchKernelGGL(treelet_refit_kernel, dim3((unsigned)grid), dim3(kRefitBlock), 0, s, H.dev,
                           (const Leaf*)leaves, nodes, nodes_c, (const uint32_t*)child, (const int32_t*)np,
                           (const int32_t*)lp,
                           (const int4*)tlist, frontier);
        hipLaunchKernelGGL(refit_top_kernel, dim3((unsigned)L.n), dim3(kTopBlock), 0, s, H.dev, nodes, nodes_c,
                           (const uint32_t*)child, (const int32_t*)np, (const int32_t*)frontier, (const int2*)top,
                           cnt);
    }
    return hipGetLastError();
}

}  // namespace bake
