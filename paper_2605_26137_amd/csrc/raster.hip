// Low-poly preparation, UV-space rasteriser, uncovered-texel fill, chart
// dilation and RGB8 encoding.
//
// The rasteriser produces the G-buffer of the paper's bake (Sec. 6.4): for
// every texel centre covered by a low-poly face in UV space, the face and the
// barycentric weights, from which the world position and the interpolated
// smooth normal follow.  Coverage is decided exactly in integers: corners are
// snapped to 1/256 texel (exact in FP32 since res is a power of two) and the
// three edge functions are evaluated in int64 at the texel centre.
#include "internal.h"

namespace bake {

namespace {

constexpr uint32_t kFaceReliable = 1u;  // UV det != 0, 3D area != 0, indices and data valid
constexpr uint32_t kFaceRaster = 2u;    // may cover texels (indices valid, UV in range, det != 0)

__device__ __forceinline__ float3 ld3(const float* p, int64_t i) {
    return make_float3(p[3 * i], p[3 * i + 1], p[3 * i + 2]);
}
__device__ __forceinline__ float3 sub3(float3 a, float3 b) {
    return make_float3(a.x - b.x, a.y - b.y, a.z - b.z);
}
__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ bool finite3(float3 a) {
    return isfinite(a.x) && isfinite(a.y) && isfinite(a.z);
}

// ---------------------------------------------------------------------------
// Low-poly preparation
// ---------------------------------------------------------------------------

// Per face: snapped UV corners, tangent T_f = sgn(det) (e1 dv2 - e2 dv1) and
// handedness h_f = sign(((e1 x e2) x T_f) . B_f) with B_f = sgn(det)(e2 du1 -
// e1 du2); reliability flags; vertex degrees for the vertex -> face CSR.
__global__ __launch_bounds__(256) void lo_face_kernel(Batch Bt, float4* __restrict__ face_t,
                                                      int4* __restrict__ face_uv,
                                                      uint32_t* __restrict__ deg) {
    int64_t lb;
    const AssetDev& As = Bt.A[block_asset(Bt, kGLoF, blockIdx.x, &lb)];
    const int64_t f = lb * 256 + threadIdx.x;
    if (f >= As.nlf) return;
    const float* __restrict__ V = As.lo_V;
    const int32_t* __restrict__ F = As.lo_F;
    const float* __restrict__ UV = As.lo_UV;
    const int64_t nv = As.nlv;
    int32_t a = F[3 * f], b = F[3 * f + 1], c = F[3 * f + 2];
    bool idx_ok = a >= 0 && b >= 0 && c >= 0 && a < nv && b < nv && c < nv;
    uint32_t st = 0;
    if (!idx_ok) st |= kStLoIndex;
    float u[6];
    bool uv_ok = true;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        u[k] = UV[6 * f + k];
        uv_ok = uv_ok && isfinite(u[k]) && u[k] >= -1.0f && u[k] <= 2.0f;
    }
    if (!uv_ok) st |= kStBadUV;
    const float sc = (float)As.res * 256.0f;
    int32_t X[3], Y[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        X[k] = uv_ok ? (int32_t)rintf(u[2 * k] * sc) : 0;
        Y[k] = uv_ok ? (int32_t)rintf(u[2 * k + 1] * sc) : 0;
    }
    int64_t du1 = X[1] - X[0], dv1 = Y[1] - Y[0], du2 = X[2] - X[0], dv2 = Y[2] - Y[0];
    int64_t det = du1 * dv2 - du2 * dv1;
    float sg = det > 0 ? 1.0f : (det < 0 ? -1.0f : 0.0f);
    float4 T4 = make_float4(0.f, 0.f, 0.f, 1.f);
    bool rel = false;
    if (idx_ok) {
        float3 A = ld3(V, a), B = ld3(V, b), C = ld3(V, c);
        bool fin = finite3(A) && finite3(B) && finite3(C);
        if (!fin) st |= kStNonFinite;
        float3 e1 = sub3(B, A), e2 = sub3(C, A);
        float fdu1 = (float)du1, fdv1 = (float)dv1, fdu2 = (float)du2, fdv2 = (float)dv2;
        float3 T = make_float3(sg * (e1.x * fdv2 - e2.x * fdv1), sg * (e1.y * fdv2 - e2.y * fdv1),
                               sg * (e1.z * fdv2 - e2.z * fdv1));
        float3 Bt3 = make_float3(sg * (e2.x * fdu1 - e1.x * fdu2), sg * (e2.y * fdu1 - e1.y * fdu2),
                                 sg * (e2.z * fdu1 - e1.z * fdu2));
        float3 n = cross3(e1, e2);
        float hs = dot3(cross3(n, T), Bt3);
        T4 = make_float4(T.x, T.y, T.z, hs < 0.f ? -1.f : 1.f);
        bool area = n.x != 0.f || n.y != 0.f || n.z != 0.f;
        rel = fin && uv_ok && det != 0 && area;
        atomicAdd(&deg[As.lv + a], 1u);
        atomicAdd(&deg[As.lv + b], 1u);
        atomicAdd(&deg[As.lv + c], 1u);
    }
    uint32_t flags = (rel ? kFaceReliable : 0u) | ((idx_ok && uv_ok && det != 0) ? kFaceRaster : 0u);
    const int64_t fg = As.lf + f;
    face_t[fg] = T4;
    face_uv[2 * fg] = make_int4(X[0], Y[0], X[1], Y[1]);
    face_uv[2 * fg + 1] = make_int4(X[2], Y[2], (int32_t)flags, 0);
    if (st) set_status(Bt, st);
}

// Adjacency entries hold asset-local face indices at the positions given by
// the (batch-wide) exclusive scan of the degrees.
__global__ __launch_bounds__(256) void lo_adj_kernel(Batch Bt, const uint32_t* __restrict__ off,
                                                     uint32_t* __restrict__ cur, int32_t* __restrict__ adj) {
    int64_t lb;
    const AssetDev& As = Bt.A[block_asset(Bt, kGLoF, blockIdx.x, &lb)];
    const int64_t f = lb * 256 + threadIdx.x;
    if (f >= As.nlf) return;
    const int32_t* __restrict__ F = As.lo_F;
    const int64_t nv = As.nlv;
    int32_t v[3] = {F[3 * f], F[3 * f + 1], F[3 * f + 2]};
    if (v[0] < 0 || v[1] < 0 || v[2] < 0 || v[0] >= nv || v[1] >= nv || v[2] >= nv) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int64_t g = As.lv + v[k];
        uint32_t slot = atomicAdd(&cur[g], 1u);
        adj[off[g] + slot] = (int32_t)f;
    }
}

// Per vertex: sort its incident faces ascending (fixed summation order, so the
// result does not depend on the order the adjacency was filled in), then
// n_v = normalise(sum (V1 - V0) x (V2 - V0)).
__global__ __launch_bounds__(256) void lo_normal_kernel(Batch Bt, const uint32_t* __restrict__ off,
                                                        int32_t* __restrict__ adj,
                                                        float4* __restrict__ lo_n) {
    int64_t lb;
    const AssetDev& As = Bt.A[block_asset(Bt, kGLoV, blockIdx.x, &lb)];
    const int64_t v = lb * 256 + threadIdx.x;
    if (v >= As.nlv) return;
    const float* __restrict__ V = As.lo_V;
    const int32_t* __restrict__ F = As.lo_F;
    const int64_t g = As.lv + v;
    uint32_t b = off[g], e = off[g + 1];
    for (uint32_t i = b + 1; i < e; ++i) {
        int32_t x = adj[i];
        uint32_t j = i;
        while (j > b && adj[j - 1] > x) {
            adj[j] = adj[j - 1];
            --j;
        }
        adj[j] = x;
    }
    float3 s = make_float3(0.f, 0.f, 0.f);
    for (uint32_t i = b; i < e; ++i) {
        int32_t f = adj[i];
        float3 A = ld3(V, F[3 * f]), B = ld3(V, F[3 * f + 1]), C = ld3(V, F[3 * f + 2]);
        float3 c = cross3(sub3(B, A), sub3(C, A));
        s.x += c.x;
        s.y += c.y;
        s.z += c.z;
    }
    float l2 = dot3(s, s);
    float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
    if (l2 > 0.f && isfinite(l2)) {
        float r = 1.0f / sqrtf(l2);
        out = make_float4(s.x * r, s.y * r, s.z * r, 1.f);
    }
    lo_n[g] = out;
}

// ---------------------------------------------------------------------------
// Rasteriser: one wave (64 lanes) per face, lanes stride over the face's
// texel bounding box.
// ---------------------------------------------------------------------------

struct FaceBox {
    int32_t X[3], Y[3];
    int32_t i0, j0, w, h;
    bool ok;
};

__device__ __forceinline__ int32_t floor_div256(int32_t x) { return x >> 8; }  // arithmetic shift

__device__ __forceinline__ FaceBox load_face_box(const int4* __restrict__ face_uv, int64_t fg,
                                                 int32_t res) {
    FaceBox fb;
    int4 p = face_uv[2 * fg], q = face_uv[2 * fg + 1];
    fb.X[0] = p.x; fb.Y[0] = p.y; fb.X[1] = p.z; fb.Y[1] = p.w; fb.X[2] = q.x; fb.Y[2] = q.y;
    fb.ok = (q.z & kFaceRaster) != 0;
    int32_t xmin = min(min(fb.X[0], fb.X[1]), fb.X[2]), xmax = max(max(fb.X[0], fb.X[1]), fb.X[2]);
    int32_t ymin = min(min(fb.Y[0], fb.Y[1]), fb.Y[2]), ymax = max(max(fb.Y[0], fb.Y[1]), fb.Y[2]);
    // texel centres 256 j + 128 inside [xmin, xmax]
    int32_t j0 = floor_div256(xmin - 128 + 255), j1 = floor_div256(xmax - 128);
    int32_t i0 = floor_div256(ymin - 128 + 255), i1 = floor_div256(ymax - 128);
    j0 = max(j0, 0); i0 = max(i0, 0);
    j1 = min(j1, res - 1); i1 = min(i1, res - 1);
    fb.j0 = j0; fb.i0 = i0;
    fb.w = j1 - j0 + 1; fb.h = i1 - i0 + 1;
    if (fb.w <= 0 || fb.h <= 0) fb.ok = false;
    return fb;
}

// Edge functions of the edges opposite corners 0, 1, 2 at texel (i, j).
__device__ __forceinline__ bool cover(const FaceBox& fb, int32_t i, int32_t j, int64_t E[3],
                                      int64_t* S) {
    int64_t cx = 256 * (int64_t)j + 128, cy = 256 * (int64_t)i + 128;
    const int32_t* X = fb.X;
    const int32_t* Y = fb.Y;
    E[0] = (int64_t)(X[2] - X[1]) * (cy - Y[1]) - (int64_t)(Y[2] - Y[1]) * (cx - X[1]);
    E[1] = (int64_t)(X[0] - X[2]) * (cy - Y[2]) - (int64_t)(Y[0] - Y[2]) * (cx - X[2]);
    E[2] = (int64_t)(X[1] - X[0]) * (cy - Y[0]) - (int64_t)(Y[1] - Y[0]) * (cx - X[0]);
    *S = E[0] + E[1] + E[2];
    bool in = (E[0] >= 0 && E[1] >= 0 && E[2] >= 0) || (E[0] <= 0 && E[1] <= 0 && E[2] <= 0);
    return in && *S != 0;
}

constexpr int kRasterBlock = 256;
constexpr int kWavesPerBlock = kRasterBlock / 64;

// The face of a raster wave, or -1 past the asset's faces.
__device__ __forceinline__ int64_t raster_face(const Batch& Bt, const AssetDev** As) {
    int64_t lb;
    *As = &Bt.A[block_asset(Bt, kGLoFWave, blockIdx.x, &lb)];
    const int64_t f = lb * kWavesPerBlock + (threadIdx.x >> 6);
    return f < (*As)->nlf ? f : -1;
}

__global__ __launch_bounds__(kRasterBlock) void raster_claim_kernel(Batch Bt, const int4* __restrict__ face_uv,
                                                                    uint32_t* __restrict__ facemap) {
    const AssetDev* As;
    const int64_t f = raster_face(Bt, &As);
    const int lane = threadIdx.x & 63;
    if (f < 0) return;
    const int32_t res = As->res;
    FaceBox fb = load_face_box(face_uv, As->lf + f, res);
    if (!fb.ok) return;
    uint32_t* fm = facemap + As->tex;
    int64_t total = (int64_t)fb.w * fb.h;
    for (int64_t k = lane; k < total; k += 64) {
        int32_t i = fb.i0 + (int32_t)(k / fb.w), j = fb.j0 + (int32_t)(k % fb.w);
        int64_t E[3], S;
        if (cover(fb, i, j, E, &S)) atomicMin(&fm[(int64_t)i * res + j], (uint32_t)f);
    }
}

__global__ __launch_bounds__(kRasterBlock) void raster_count_kernel(Batch Bt, const int4* __restrict__ face_uv,
                                                                    const uint32_t* __restrict__ facemap,
                                                                    uint32_t* __restrict__ cnt) {
    const AssetDev* As;
    const int64_t f = raster_face(Bt, &As);
    const int lane = threadIdx.x & 63;
    if (f < 0) return;
    const int32_t res = As->res;
    FaceBox fb = load_face_box(face_uv, As->lf + f, res);
    const uint32_t* fm = facemap + As->tex;
    uint32_t c = 0;
    if (fb.ok) {
        int64_t total = (int64_t)fb.w * fb.h;
        for (int64_t k0 = 0; k0 < total; k0 += 64) {
            int64_t k = k0 + lane;
            bool win = false;
            if (k < total) {
                int32_t i = fb.i0 + (int32_t)(k / fb.w), j = fb.j0 + (int32_t)(k % fb.w);
                int64_t E[3], S;
                win = cover(fb, i, j, E, &S) && fm[(int64_t)i * res + j] == (uint32_t)f;
            }
            c += (uint32_t)__popcll(__ballot(win));
        }
    }
    if (lane == 0) cnt[As->lf + f] = c;
}

__global__ __launch_bounds__(kRasterBlock) void raster_emit_kernel(Batch Bt, const int4* __restrict__ face_uv,
                                                                   const uint32_t* __restrict__ facemap,
                                                                   const uint32_t* __restrict__ off,
                                                                   Ray* __restrict__ rays) {
    const AssetDev* As;
    const int64_t f = raster_face(Bt, &As);
    const int lane = threadIdx.x & 63;
    if (f < 0) return;
    const int32_t res = As->res;
    FaceBox fb = load_face_box(face_uv, As->lf + f, res);
    if (!fb.ok) return;
    const uint32_t* fm = facemap + As->tex;
    int64_t total = (int64_t)fb.w * fb.h;
    uint32_t run = off[As->lf + f];
    for (int64_t k0 = 0; k0 < total; k0 += 64) {
        int64_t k = k0 + lane;
        bool win = false;
        int64_t E[3] = {0, 0, 0}, S = 1;
        int32_t i = 0, j = 0;
        if (k < total) {
            i = fb.i0 + (int32_t)(k / fb.w);
            j = fb.j0 + (int32_t)(k % fb.w);
            win = cover(fb, i, j, E, &S) && fm[(int64_t)i * res + j] == (uint32_t)f;
        }
        uint64_t m = __ballot(win);
        if (win) {
            uint32_t r = run + (uint32_t)__popcll(m & __lanemask_lt());
            Ray ray;
            ray.texel = i * res + j;
            ray.face = (int32_t)f;
            float fs = (float)S;
            ray.b1 = (float)E[1] / fs;
            ray.b2 = (float)E[2] / fs;
            rays[r] = ray;
        }
        run += (uint32_t)__popcll(m);
    }
}

// ---------------------------------------------------------------------------
// Uncovered texels, dilation, RGB8
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void fill_uncovered_kernel(Batch Bt, const uint32_t* __restrict__ facemap,
                                                             uint8_t* __restrict__ level) {
    int64_t lb;
    const AssetDev& As = Bt.A[block_asset(Bt, kGTex, blockIdx.x, &lb)];
    const int64_t t = lb * 256 + threadIdx.x;
    if (t >= (int64_t)As.res * As.res) return;
    bool cov = facemap[As.tex + t] != 0x7FFFFFFFu;
    level[As.tex + t] = cov ? 0 : 255;
    if (!cov) {
        As.out_map[3 * t] = 0.f;
        As.out_map[3 * t + 1] = 0.f;
        As.out_map[3 * t + 2] = 1.f;
        As.out_hit[t] = kUncovered;
    }
}

// The uncovered texels alone (no dilation): (0,0,1) and the uncovered status.
__global__ __launch_bounds__(256) void uncovered_kernel(Batch Bt, const uint32_t* __restrict__ facemap) {
    int64_t lb;
    const AssetDev& As = Bt.A[block_asset(Bt, kGTex, blockIdx.x, &lb)];
    const int64_t t = lb * 256 + threadIdx.x;
    if (t >= (int64_t)As.res * As.res || facemap[As.tex + t] != 0x7FFFFFFFu) return;
    As.out_map[3 * t] = 0.f;
    As.out_map[3 * t + 1] = 0.f;
    As.out_map[3 * t + 2] = 1.f;
    As.out_hit[t] = kUncovered;
}

// Pass k: a still-empty texel takes the normalised sum of its 8 neighbours
// that had a value before this pass (level < k).  Texels written in this pass
// are never read in it, so the map is updated in place.
__global__ __launch_bounds__(256) void dilate_kernel(Batch Bt, int pass, uint8_t* __restrict__ level_all) {
    int64_t lb;
    const AssetDev& As = Bt.A[block_asset(Bt, kGTex, blockIdx.x, &lb)];
    const int32_t res = As.res;
    const int64_t t = lb * 256 + threadIdx.x;
    if (t >= (int64_t)res * res) return;
    uint8_t* __restrict__ level = level_all + As.tex;
    float* __restrict__ map = As.out_map;
    if (level[t] != 255) return;
    const int32_t i = (int32_t)(t >> As.log2res), j = (int32_t)(t & (res - 1));
    float sx = 0.f, sy = 0.f, sz = 0.f;
    int cnt = 0;
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj) {
            if (di == 0 && dj == 0) continue;
            int32_t ii = i + di, jj = j + dj;
            if (ii < 0 || jj < 0 || ii >= res || jj >= res) continue;
            int64_t u = (int64_t)ii * res + jj;
            if (level[u] < pass) {
                sx += map[3 * u];
                sy += map[3 * u + 1];
                sz += map[3 * u + 2];
                ++cnt;
            }
        }
    }
    if (cnt == 0) return;
    float l2 = sx * sx + sy * sy + sz * sz;
    if (!(l2 > 0.f)) return;
    float r = 1.0f / sqrtf(l2);
    map[3 * t] = sx * r;
    map[3 * t + 1] = sy * r;
    map[3 * t + 2] = sz * r;
    level[t] = (uint8_t)pass;
}

// Uncovered fill and 1 <= k <= kMaxFusedPasses dilation passes in one launch.
// A workgroup takes a kFinishTile^2 texel tile plus a k-texel halo, R = tile
// + 2k <= 64 texels a side: one wave per region row at a time, one lane per
// column.  The region's values go to LDS (covered texels with their traced
// value, uncovered ones as (0,0,1)) and its rows to 64-bit masks: inside the
// image, and has a value before the pass (covered, or filled in an earlier
// pass).  A pass fills, with the pass rule of dilate_kernel, only the empty
// texels that the masks show to have a valued neighbour; the others read
// nothing.  A value at distance d from the region's edge is exact through
// pass d, so the tile (d >= k) is exact after k passes: the result is bitwise
// that of the fill + per-pass launches (same neighbours, same order of sums).
constexpr int kFinishBlock = 512;
constexpr int kFinishWaves = kFinishBlock / 64;
static_assert(kFinishTile + 2 * kMaxFusedPasses <= 64, "a region row fits one wave");

template <int PASSES>
__global__ __launch_bounds__(kFinishBlock) void finish_kernel(Batch Bt, const uint32_t* __restrict__ facemap_all) {
    static_assert(PASSES >= 1 && PASSES <= kMaxFusedPasses, "fused pass count");
    constexpr int R = kFinishTile + 2 * PASSES;                // region side
    constexpr int kRows = (R + kFinishWaves - 1) / kFinishWaves;  // region rows per wave
    __shared__ float s_map[R][64][3];
    __shared__ uint64_t s_in[R], s_val[2][R];
    int64_t lt;
    const AssetDev& As = Bt.A[block_asset(Bt, kGTile, blockIdx.x, &lt)];
    const int32_t res = As.res;
    const int32_t tiles_x = (res + kFinishTile - 1) / kFinishTile;
    const int32_t oi = (int32_t)(lt / tiles_x) * kFinishTile - PASSES;  // region origin
    const int32_t oj = (int32_t)(lt % tiles_x) * kFinishTile - PASSES;
    const uint32_t* __restrict__ facemap = facemap_all + As.tex;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t j = oj + lane;
    const bool col_in = lane < R && j >= 0 && j < res;
    // Loads of all the wave's rows first: coverage, then the map values of
    // the covered texels (two load latencies per wave).
    int32_t t[kRows];
    bool cov[kRows];
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
        const int r = wave + u * kFinishWaves;
        const int32_t i = oi + r;
        const bool in = r < R && col_in && i >= 0 && i < res;
        t[u] = in ? i * res + j : -1;
        cov[u] = in && facemap[t[u]] != 0x7FFFFFFFu;
    }
    float m0[kRows], m1[kRows], m2[kRows];
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
        m0[u] = 0.f;
        m1[u] = 0.f;
        m2[u] = 1.f;
        if (cov[u]) {
            m0[u] = As.out_map[3 * t[u]];
            m1[u] = As.out_map[3 * t[u] + 1];
            m2[u] = As.out_map[3 * t[u] + 2];
        }
    }
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
        const int r = wave + u * kFinishWaves;
        if (r >= R) break;  // wave-uniform
        s_map[r][lane][0] = m0[u];
        s_map[r][lane][1] = m1[u];
        s_map[r][lane][2] = m2[u];
        const uint64_t bin = __ballot(t[u] >= 0), bcov = __ballot(cov[u]);
        if (lane == 0) {
            s_in[r] = bin;
            s_val[0][r] = bcov;
        }
    }
    __syncthreads();
    for (int pass = 1; pass <= PASSES; ++pass) {
        const uint64_t* cur = s_val[(pass - 1) & 1];
        uint64_t* nxt = s_val[pass & 1];
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
            const int r = wave + u * kFinishWaves;
            if (r >= R) break;  // wave-uniform
            const uint64_t vu = r > 0 ? cur[r - 1] : 0ull, vc = cur[r], vd = r + 1 < R ? cur[r + 1] : 0ull;
            const uint64_t vm = vu | vc | vd;
            const uint64_t cand = (vm | (vm << 1) | (vm >> 1)) & s_in[r] & ~vc;
            bool filled = false;
            if ((cand >> lane) & 1ull) {
                float sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
                for (int di = -1; di <= 1; ++di) {
                    const uint64_t row = di < 0 ? vu : (di == 0 ? vc : vd);
#pragma unroll
                    for (int dj = -1; dj <= 1; ++dj) {
                        if (di == 0 && dj == 0) continue;
                        const int ii = r + di, jj = lane + dj;
                        if (ii < 0 || jj < 0 || ii >= R || jj >= R) continue;
                        if ((row >> jj) & 1ull) {
                            sx += s_map[ii][jj][0];
                            sy += s_map[ii][jj][1];
                            sz += s_map[ii][jj][2];
                        }
                    }
                }
                // at least one neighbour had a value (the candidate mask)
                const float l2 = sx * sx + sy * sy + sz * sz;
                if (l2 > 0.f) {
                    const float inv = 1.0f / sqrtf(l2);
                    s_map[r][lane][0] = sx * inv;
                    s_map[r][lane][1] = sy * inv;
                    s_map[r][lane][2] = sz * inv;
                    filled = true;
                }
            }
            // texels filled in this pass are read by no one in it: the pass
            // reads the masks of `cur` and writes those of `nxt`
            const uint64_t bf = __ballot(filled);
            if (lane == 0) nxt[r] = vc | bf;
        }
        __syncthreads();
    }
    // the tile's uncovered texels, filled or (0,0,1)
    const bool col_tile = lane >= PASSES && lane < PASSES + kFinishTile;
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
        const int r = wave + u * kFinishWaves;
        if (r < PASSES || r >= PASSES + kFinishTile || !col_tile || t[u] < 0 || cov[u]) continue;
        As.out_map[3 * t[u]] = s_map[r][lane][0];
        As.out_map[3 * t[u] + 1] = s_map[r][lane][1];
        As.out_map[3 * t[u] + 2] = s_map[r][lane][2];
        As.out_hit[t[u]] = kUncovered;
    }
}

__global__ __launch_bounds__(256) void rgb8_kernel(Batch Bt) {
    int64_t lb;
    const AssetDev& As = Bt.A[block_asset(Bt, kGTex3, blockIdx.x, &lb)];
    const int64_t k = lb * 256 + threadIdx.x;
    if (!As.out_rgb8 || k >= 3 * (int64_t)As.res * As.res) return;
    float c = floorf((As.out_map[k] + 1.0f) * 127.5f + 0.5f);
    c = fminf(fmaxf(c, 0.0f), 255.0f);
    As.out_rgb8[k] = (uint8_t)c;
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_lo_prep(const BatchHost& H, hipStream_t s) {
    const Layout& L = H.L;
    char* ws = H.ws;
    uint32_t* deg = (uint32_t*)(ws + L.lo_deg);
    uint32_t* off = (uint32_t*)(ws + L.lo_off);
    uint32_t* cur = (uint32_t*)(ws + L.lo_cur);
    hipError_t e;
    if ((e = fill_u32(deg, 0, L.t_lv, s)) != hipSuccess) return e;
    if ((e = fill_u32(cur, 0, L.t_lv, s)) != hipSuccess) return e;
    if (H.blocks(kGLoF) > 0) {
        hipLaunchKernelGGL(lo_face_kernel, dim3((unsigned)H.blocks(kGLoF)), dim3(256), 0, s, H.dev,
                           (float4*)(ws + L.face_t), (int4*)(ws + L.face_uv), deg);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // batch-wide scan: vertex g's faces sit at [off[g], off[g + 1])
    if ((e = exclusive_scan_u32(deg, off, L.t_lv, (uint32_t*)(ws + L.scan_tmp), off + L.t_lv, s)) !=
        hipSuccess)
        return e;
    if (H.blocks(kGLoF) > 0) {
        hipLaunchKernelGGL(lo_adj_kernel, dim3((unsigned)H.blocks(kGLoF)), dim3(256), 0, s, H.dev,
                           (const uint32_t*)off, cur, (int32_t*)(ws + L.lo_adj));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (H.blocks(kGLoV) > 0) {
        hipLaunchKernelGGL(lo_normal_kernel, dim3((unsigned)H.blocks(kGLoV)), dim3(256), 0, s, H.dev,
                           (const uint32_t*)off, (int32_t*)(ws + L.lo_adj), (float4*)(ws + L.lo_n));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_raster(const BatchHost& H, hipStream_t s) {
    const Layout& L = H.L;
    char* ws = H.ws;
    uint32_t* facemap = (uint32_t*)(ws + L.facemap);
    uint32_t* cnt = (uint32_t*)(ws + L.face_cnt);
    uint32_t* off = (uint32_t*)(ws + L.face_off);
    const int4* fuv = (const int4*)(ws + L.face_uv);
    hipError_t e;
    if ((e = fill_u32(facemap, 0x7FFFFFFFu, L.t_tex, s)) != hipSuccess) return e;
    const unsigned g = (unsigned)H.blocks(kGLoFWave);
    if (g > 0) {
        hipLaunchKernelGGL(raster_claim_kernel, dim3(g), dim3(kRasterBlock), 0, s, H.dev, fuv, facemap);
        hipLaunchKernelGGL(raster_count_kernel, dim3(g), dim3(kRasterBlock), 0, s, H.dev, fuv,
                           (const uint32_t*)facemap, cnt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // batch-wide scan: the face-ordered ray lists of the assets, concatenated
    if ((e = exclusive_scan_u32(cnt, off, L.t_lf, (uint32_t*)(ws + L.scan_tmp), off + L.t_lf, s)) !=
        hipSuccess)
        return e;
    if ((e = launch_ray_spaces(H, s)) != hipSuccess) return e;
    if (g > 0) {
        hipLaunchKernelGGL(raster_emit_kernel, dim3(g), dim3(kRasterBlock), 0, s, H.dev, fuv,
                           (const uint32_t*)facemap, (const uint32_t*)off, (Ray*)(ws + L.rays));
    }
    return hipGetLastError();
}

hipError_t launch_fill_uncovered(const BatchHost& H, hipStream_t s) {
    if (H.blocks(kGTex) == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_uncovered_kernel, dim3((unsigned)H.blocks(kGTex)), dim3(256), 0, s, H.dev,
                       (const uint32_t*)(H.ws + H.L.facemap), (uint8_t*)(H.ws + H.L.level));
    return hipGetLastError();
}

// After the traversal: uncovered fill and dilation, fused for few passes.
hipError_t launch_dilate(const BatchHost& H, int passes, hipStream_t s) {
    const uint32_t* fm = (const uint32_t*)(H.ws + H.L.facemap);
    if (passes == 0) {
        if (H.blocks(kGTex) == 0) return hipSuccess;
        hipLaunchKernelGGL(uncovered_kernel, dim3((unsigned)H.blocks(kGTex)), dim3(256), 0, s, H.dev, fm);
        return hipGetLastError();
    }
    if (passes <= kMaxFusedPasses) {
        if (H.blocks(kGTile) == 0) return hipSuccess;
        const dim3 grid((unsigned)H.blocks(kGTile)), block(kFinishBlock);
        switch (passes) {
            case 1: hipLaunchKernelGGL(finish_kernel<1>, grid, block, 0, s, H.dev, fm); break;
            case 2: hipLaunchKernelGGL(finish_kernel<2>, grid, block, 0, s, H.dev, fm); break;
            case 3: hipLaunchKernelGGL(finish_kernel<3>, grid, block, 0, s, H.dev, fm); break;
            default: hipLaunchKernelGGL(finish_kernel<4>, grid, block, 0, s, H.dev, fm); break;
        }
        static_assert(kMaxFusedPasses == 4, "one finish_kernel instance per fused pass count");
        return hipGetLastError();
    }
    hipError_t e = launch_fill_uncovered(H, s);
    if (e != hipSuccess || H.blocks(kGTex) == 0) return e;
    for (int k = 1; k <= passes; ++k) {
        hipLaunchKernelGGL(dilate_kernel, dim3((unsigned)H.blocks(kGTex)), dim3(256), 0, s, H.dev, k,
                           (uint8_t*)(H.ws + H.L.level));
    }
    return hipGetLastError();
}

hipError_t launch_rgb8(const BatchHost& H, hipStream_t s) {
    if (H.blocks(kGTex3) == 0) return hipSuccess;
    hipLaunchKernelGGL(rgb8_kernel, dim3((unsigned)H.blocks(kGTex3)), dim3(256), 0, s, H.dev);
    return hipGetLastError();
}

}  // namespace bake
