// Hidden-face removal (Sec. 6.2), second half: the flood fill.  Seeds are the
// faces some camera ray hit first; an exterior face f promotes a face g that
// shares an edge with it (two distinct vertex indices in common) when their
// normals agree in direction, n_f . n_g > 0 with n = (V1 - V0) x (V2 - V0).
// The sign is taken in FP64 from the float vertices with no fused
// operations, in a fixed order (x, y, z), so it is the same decision
// wherever it is evaluated.  The condition is symmetric, so the exterior is
// the set of faces joined to a seed by such edges; the traversal order (and
// the order of the per-vertex face lists, filled with atomics) does not
// change it.
//
// Layout: per-vertex face lists (CSR: deg -> off by a scan, adj filled with
// per-vertex cursors), u32 flags ext[n_f], two frontier lists of face ids.
// The breadth-first expansion runs in one workgroup (the paper's meshes have
// about 22K faces): each level walks the frontier's faces' vertex lists,
// claims newly promoted faces with an atomic exchange on their flag and
// appends them to the next frontier; the loop ends when a level adds no face
// (at most n_f levels).
#include "internal.h"

namespace bake {

namespace {

constexpr int kFillBlock = 1024;

__device__ __forceinline__ bool face_verts(const AssetDev& As, int64_t f, int32_t v[3]) {
    v[0] = As.hi_F[3 * f];
    v[1] = As.hi_F[3 * f + 1];
    v[2] = As.hi_F[3 * f + 2];
    return v[0] >= 0 && v[1] >= 0 && v[2] >= 0 && v[0] < As.nhv && v[1] < As.nhv && v[2] < As.nhv;
}

struct d3 {
    double x, y, z;
};

__device__ __forceinline__ d3 face_normal(const AssetDev& As, const int32_t v[3]) {
#pragma clang fp contract(off)
    const float* V = As.hi_V;
    const double ax = V[3 * (int64_t)v[0]], ay = V[3 * (int64_t)v[0] + 1], az = V[3 * (int64_t)v[0] + 2];
    const double bx = (double)V[3 * (int64_t)v[1]] - ax, by = (double)V[3 * (int64_t)v[1] + 1] - ay,
                 bz = (double)V[3 * (int64_t)v[1] + 2] - az;
    const double cx = (double)V[3 * (int64_t)v[2]] - ax, cy = (double)V[3 * (int64_t)v[2] + 1] - ay,
                 cz = (double)V[3 * (int64_t)v[2] + 2] - az;
    d3 n;
    n.x = by * cz - bz * cy;
    n.y = bz * cx - bx * cz;
    n.z = bx * cy - by * cx;
    return n;
}

__device__ __forceinline__ bool agree(const d3& a, const d3& b) {
#pragma clang fp contract(off)
    const double d = a.x * b.x + a.y * b.y + a.z * b.z;
    return d > 0.0;
}

__global__ __launch_bounds__(256) void fv_count_kernel(Batch B, uint32_t* __restrict__ deg) {
    const AssetDev& As = B.A[0];
    const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (f >= As.nhf) return;
    int32_t v[3];
    if (!face_verts(As, f, v)) {
        set_status(B, kStHiIndex);
        return;
    }
    for (int i = 0; i < 3; ++i)
        if ((i < 1 || v[i] != v[0]) && (i < 2 || v[i] != v[1])) atomicAdd(&deg[v[i]], 1u);
}

__global__ __launch_bounds__(256) void fv_fill_kernel(Batch B, const uint32_t* __restrict__ off,
                                                      uint32_t* __restrict__ cur, uint32_t* __restrict__ adj) {
    const AssetDev& As = B.A[0];
    const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (f >= As.nhf) return;
    int32_t v[3];
    if (!face_verts(As, f, v)) return;
    for (int i = 0; i < 3; ++i)
        if ((i < 1 || v[i] != v[0]) && (i < 2 || v[i] != v[1])) adj[off[v[i]] + atomicAdd(&cur[v[i]], 1u)] = (uint32_t)f;
}

// Distinct vertex indices f and g share (f's vertices in fv).
__device__ __forceinline__ int shared_count(const int32_t fv[3], const int32_t gv[3]) {
    int n = 0;
    for (int i = 0; i < 3; ++i) {
        if ((i >= 1 && fv[i] == fv[0]) || (i >= 2 && fv[i] == fv[1])) continue;
        n += (gv[0] == fv[i] || gv[1] == fv[i] || gv[2] == fv[i]) ? 1 : 0;
    }
    return n;
}

__global__ __launch_bounds__(kFillBlock) void flood_fill_kernel(Batch B, FillRun r) {
    __shared__ uint32_t s_n[2];
    const AssetDev& As = B.A[0];
    const int64_t nf = As.nhf;
    if (threadIdx.x == 0) s_n[0] = s_n[1] = 0;
    __syncthreads();
    for (int64_t f = threadIdx.x; f < nf; f += kFillBlock) {
        const uint32_t e = r.visible[f] ? 1u : 0u;
        r.ext[f] = e;
        if (e) r.front0[atomicAdd(&s_n[0], 1u)] = (uint32_t)f;
    }
    __syncthreads();
    int c = 0;
    uint32_t count = s_n[0];
    // every level with a non-empty frontier promotes its frontier's faces for
    // good, so there are at most nf levels
    for (int64_t level = 0; count > 0 && level <= nf; ++level) {
        const uint32_t* front = c == 0 ? r.front0 : r.front1;
        uint32_t* next = c == 0 ? r.front1 : r.front0;
        if (threadIdx.x == 0) s_n[1 - c] = 0;
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < count; k += kFillBlock) {
            const int64_t f = front[k];
            int32_t fv[3];
            if (!face_verts(As, f, fv)) continue;
            const d3 nf_ = face_normal(As, fv);
            for (int i = 0; i < 3; ++i) {
                if ((i >= 1 && fv[i] == fv[0]) || (i >= 2 && fv[i] == fv[1])) continue;
                for (uint32_t e = r.off[fv[i]]; e < r.off[fv[i] + 1]; ++e) {
                    const int64_t g = r.adj[e];
                    if (g == f || r.ext[g]) continue;
                    int32_t gv[3];
                    if (!face_verts(As, g, gv) || shared_count(fv, gv) < 2) continue;
                    if (!agree(nf_, face_normal(As, gv))) continue;
                    if (atomicExch(&r.ext[g], 1u) == 0u) next[atomicAdd(&s_n[1 - c], 1u)] = (uint32_t)g;
                }
            }
        }
        __syncthreads();
        count = s_n[1 - c];
        c = 1 - c;
        __syncthreads();
    }
    if (count > 0) set_status(B, kStInternal);  // only a corrupted list gets here
    for (int64_t f = threadIdx.x; f < nf; f += kFillBlock) {
        if (r.visible_out) r.visible_out[f] = r.visible[f] ? 1 : 0;
        if (r.exterior_out) r.exterior_out[f] = r.ext[f] ? 1 : 0;
    }
}

}  // namespace

hipError_t launch_flood_fill(const BatchHost& H, const FillRun& r, hipStream_t s) {
    const AssetDev& As = H.A[0];
    const int64_t nf = As.nhf, nv = As.nhv;
    hipError_t e;
    if ((e = fill_u32(r.deg, 0, nv + 1, s)) != hipSuccess) return e;
    if ((e = fill_u32(r.cur, 0, nv + 1, s)) != hipSuccess) return e;
    const unsigned g = (unsigned)((nf + 255) / 256);
    if (g > 0) hipLaunchKernelGGL(fv_count_kernel, dim3(g), dim3(256), 0, s, H.dev, r.deg);
    if ((e = exclusive_scan_u32(r.deg, r.off, nv, r.scan_tmp, r.off + nv, s)) != hipSuccess) return e;
    if (g > 0) hipLaunchKernelGGL(fv_fill_kernel, dim3(g), dim3(256), 0, s, H.dev, (const uint32_t*)r.off, r.cur, r.adj);
    hipLaunchKernelGGL(flood_fill_kernel, dim3(1), dim3(kFillBlock), 0, s, H.dev, r);
    return hipGetLastError();
}

}  // namespace bake
