// Backward of a loss on the baked map (pre-dilation), with the texel -> face
// assignment, the barycentrics, the hit triangle and the UV handedness held
// fixed.  Differentiable inputs: low-poly positions lo_V (through the texel
// position p, the area-weighted vertex normals and the face tangent T_f) and
// the high-poly normals hi_N (through the interpolated hit normal).
//
// Per ray (forward):  p = sum b_k V_k,  m = sum b_k n_k,  d = m/|m|;
//   p + t d = A + beta1 (B - A) + beta2 (C - A) on the hit triangle's plane;
//   h = sum beta_k N_k, n = h/|h|;  T~ = T_f - (d.T_f) d, T' = T~/|T~|,
//   B' = h_f (d x T');  out = (n.T', n.B', n.d).
// The adjoint walks this chain backwards per ray, then reduces:
//   * low-poly: rays are contiguous per face in the ray list, so one wave per
//     face sums its rays (lane-strided, then a fixed shuffle tree); vertices
//     gather their faces through the ascending vertex -> face adjacency, the
//     normalisation and the face cross products are differentiated, and a
//     second gather finishes dL/dlo_V;
//   * high-poly: each hit ray contributes beta_k h_bar to the three vertices
//     of its triangle; the (vertex, ray*3 + corner) pairs are radix-sorted
//     stably and each vertex sums its run in ray order.
// No floating-point atomics: the result is bitwise reproducible.  In a batch
// the per-ray kernels take (asset, 64-ray batch) items like the traversal,
// and the reductions stay inside each asset's ranges.
#include <algorithm>

#include "internal.h"

namespace bake {

namespace {

__device__ __forceinline__ float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ __forceinline__ float3 add3(float3 a, float3 b) { return f3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 sub3(float3 a, float3 b) { return f3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 mul3(float3 a, float s) { return f3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return f3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float3 ld3(const float* p, int64_t i) {
    return f3(p[3 * i], p[3 * i + 1], p[3 * i + 2]);
}
__device__ __forceinline__ void st3(float* p, int64_t i, float3 v) {
    p[3 * i] = v.x;
    p[3 * i + 1] = v.y;
    p[3 * i + 2] = v.z;
}
// (x - (x.u) u) / len: adjoint of u = y / |y| with |y| = len
__device__ __forceinline__ float3 unit_adj(float3 xb, float3 u, float len) {
    return mul3(sub3(xb, mul3(u, dot3(xb, u))), 1.0f / len);
}

struct RayGrad {  // 36 B per ray: what the low-poly chain needs
    float3 pb, mb, tfb;
};

// What the high-poly sums need of a ray, in one 32-B record: h_bar and the
// hit weights beta1, beta2 (beta0 = 1 - beta1 - beta2).
struct alignas(16) HiTerm {
    float4 a;  // h_bar.xyz, beta1
    float4 b;  // beta2, -, -, -
};
static_assert(sizeof(HiTerm) == 32, "HiTerm is 32 B");

// The (asset, 64-ray batch) item q: the asset and the wave's global ray
// (invalid when past the asset's rays).
struct RayItem {
    int a;
    int64_t r;     // global ray index
    bool valid;
    int64_t begin, end;  // the asset's global ray range
};

__device__ __forceinline__ RayItem ray_item(const Batch& B, uint32_t q, int lane) {
    RayItem it;
    it.a = upper_asset(B.rb_pf, B.n, q);
    const uint32_t nr = B.cnt[(int64_t)it.a * kCntSlots + kCntRays];
    const uint32_t k = (q - B.rb_pf[it.a]) * 64u + (uint32_t)lane;
    it.begin = B.ray_pf[it.a];
    it.end = it.begin + nr;
    it.r = it.begin + k;
    it.valid = k < nr;
    return it;
}

// Per-ray adjoint.  Also emits the three (hi vertex, item) sort pairs of the
// ray; rays without a hit emit the out-of-range key nhv.
__global__ __launch_bounds__(256) void bwd_ray_kernel(Batch B, const Ray* __restrict__ rays,
                                                      const Hit* __restrict__ hits,
                                                      const float4* __restrict__ lo_n_all,
                                                      const float4* __restrict__ face_t_all,
                                                      RayGrad* __restrict__ rg, HiTerm* __restrict__ ht,
                                                      uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    if (!sealed(B)) return;
    const int lane = threadIdx.x & 63;
    const uint32_t nb = B.rb_pf[B.n];
    const uint32_t waves = gridDim.x * 4u;
    for (uint32_t q = __builtin_amdgcn_readfirstlane(blockIdx.x * 4u + (threadIdx.x >> 6)); q < nb;
         q += waves) {
        const RayItem it = ray_item(B, q, lane);
        if (!it.valid) continue;
        const AssetDev& As = B.A[it.a];
        const int64_t r = it.r;
        const int64_t nhv = As.nhv;
        const Ray ray = rays[r];
        const Hit hit = hits[r];
        RayGrad g;
        g.pb = g.mb = g.tfb = f3(0.f, 0.f, 0.f);
        HiTerm term;
        term.a = make_float4(0.f, 0.f, 0.f, 0.f);
        term.b = make_float4(0.f, 0.f, 0.f, 0.f);
        uint32_t kv[3] = {(uint32_t)nhv, (uint32_t)nhv, (uint32_t)nhv};
        const float* grad_map = B.G[it.a].grad_map;  // NULL: the asset wants no gradient
        if (hit.id >= 0 && grad_map) {
            const float4* lo_n = lo_n_all + As.lv;
            const int32_t* lo_F = As.lo_F;
            const int32_t* hi_F = As.hi_F;
            const float* hi_V = As.hi_V;
            const float* hi_N = As.hi_N;
            const int32_t f = ray.face;
            const float b1 = ray.b1, b2 = ray.b2, b0 = 1.0f - b1 - b2;
            const int32_t i0 = lo_F[3 * f], i1 = lo_F[3 * f + 1], i2 = lo_F[3 * f + 2];
            const float4 n0 = lo_n[i0], n1 = lo_n[i1], n2 = lo_n[i2];
            const float3 m = f3(b0 * n0.x + b1 * n1.x + b2 * n2.x, b0 * n0.y + b1 * n1.y + b2 * n2.y,
                                b0 * n0.z + b1 * n1.z + b2 * n2.z);
            const float lm = sqrtf(dot3(m, m));
            const float3 d = mul3(m, 1.0f / lm);
            const float4 T4 = face_t_all[As.lf + f];
            const float3 Tf = f3(T4.x, T4.y, T4.z);
            const float H = T4.w;
            const float3 Tt = sub3(Tf, mul3(d, dot3(d, Tf)));
            const float lt = sqrtf(dot3(Tt, Tt));
            const float3 Tp = mul3(Tt, 1.0f / lt);
            const float3 Bp = mul3(cross3(d, Tp), H);
            const int32_t j0 = hi_F[3 * (int64_t)hit.id], j1 = hi_F[3 * (int64_t)hit.id + 1],
                          j2 = hi_F[3 * (int64_t)hit.id + 2];
            const float3 A = ld3(hi_V, j0), e1 = sub3(ld3(hi_V, j1), A), e2 = sub3(ld3(hi_V, j2), A);
            const float3 N0 = ld3(hi_N, j0), N1 = ld3(hi_N, j1), N2 = ld3(hi_N, j2);
            const float be1 = hit.beta1, be2 = hit.beta2, be0 = 1.0f - be1 - be2;
            const float3 h = add3(add3(mul3(N0, be0), mul3(N1, be1)), mul3(N2, be2));
            const float lh = sqrtf(dot3(h, h));
            const float3 n = mul3(h, 1.0f / lh);
            const float3 o = ld3(grad_map, ray.texel);
            // out = (n.T', n.B', n.d)
            const float3 nb3 = add3(add3(mul3(Tp, o.x), mul3(Bp, o.y)), mul3(d, o.z));
            const float3 Tpb = add3(mul3(n, o.x), mul3(cross3(n, d), o.y * H));
            float3 db = add3(mul3(n, o.z), mul3(cross3(Tp, n), o.y * H));
            // T' = T~/|T~|, T~ = T_f - (d.T_f) d
            const float3 Ttb = unit_adj(Tpb, Tp, lt);
            const float3 Tfb = sub3(Ttb, mul3(d, dot3(d, Ttb)));
            db = sub3(db, add3(mul3(Ttb, dot3(d, Tf)), mul3(Tf, dot3(d, Ttb))));
            // n = h/|h|; h = sum beta_k N_k
            const float3 hb = unit_adj(nb3, n, lh);
            const float bb1 = dot3(hb, sub3(N1, N0)), bb2 = dot3(hb, sub3(N2, N0));
            // M (t, beta1, beta2) = p - A with M = [-d | e1 | e2]:  w = M^-T (0, bb1, bb2),
            // by Cramer on M^T (columns = the rows of M)
            const float3 c0 = f3(-d.x, e1.x, e2.x), c1 = f3(-d.y, e1.y, e2.y), c2 = f3(-d.z, e1.z, e2.z);
            const float3 rhs = f3(0.f, bb1, bb2);
            const float3 c12 = cross3(c1, c2);
            const float D = dot3(c0, c12);
            const float rD = 1.0f / D;
            const float3 w = f3(dot3(rhs, c12) * rD, dot3(c0, cross3(rhs, c2)) * rD,
                                dot3(c0, cross3(c1, rhs)) * rD);
            db = add3(db, mul3(w, hit.t));
            g.pb = w;
            g.mb = unit_adj(db, d, lm);
            g.tfb = Tfb;
            term.a = make_float4(hb.x, hb.y, hb.z, be1);
            term.b = make_float4(be2, 0.f, 0.f, 0.f);
            kv[0] = (uint32_t)j0;
            kv[1] = (uint32_t)j1;
            kv[2] = (uint32_t)j2;
        }
        rg[r] = g;
        ht[r] = term;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            keys[3 * r + k] = kv[k];
            vals[3 * r + k] = (uint32_t)(3 * r + k);
        }
    }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One wave per low-poly face: sums over its rays of b_k p_bar, b_k m_bar and
// T_f_bar (lane-strided in ray order, then a fixed shuffle tree), and turns
// T_f_bar into corner contributions through T_f = c1 (V1 - V0) + c2 (V2 - V0).
// Output per face: Vbar[3 corners][3], nbar[3 corners][3].
__global__ __launch_bounds__(256) void bwd_face_kernel(Batch B, const Ray* __restrict__ rays,
                                                       const RayGrad* __restrict__ rg,
                                                       const uint32_t* __restrict__ face_off,
                                                       const int4* __restrict__ face_uv,
                                                       float* __restrict__ face_acc) {
    if (!sealed(B)) return;
    int64_t lb;
    const AssetDev& As = B.A[block_asset(B, kGLoFWave, blockIdx.x, &lb)];
    const int64_t f = lb * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (f >= As.nlf) return;
    const int64_t fg = As.lf + f;
    const uint32_t b = face_off[fg], e = face_off[fg + 1];
    float acc[21];
#pragma unroll
    for (int q = 0; q < 21; ++q) acc[q] = 0.f;
    for (uint32_t r = b + lane; r < e; r += 64) {
        const Ray ray = rays[r];
        const RayGrad g = rg[r];
        const float bk[3] = {1.0f - ray.b1 - ray.b2, ray.b1, ray.b2};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            acc[3 * k] += bk[k] * g.pb.x;
            acc[3 * k + 1] += bk[k] * g.pb.y;
            acc[3 * k + 2] += bk[k] * g.pb.z;
            acc[9 + 3 * k] += bk[k] * g.mb.x;
            acc[9 + 3 * k + 1] += bk[k] * g.mb.y;
            acc[9 + 3 * k + 2] += bk[k] * g.mb.z;
        }
        acc[18] += g.tfb.x;
        acc[19] += g.tfb.y;
        acc[20] += g.tfb.z;
    }
#pragma unroll
    for (int q = 0; q < 21; ++q) acc[q] = wave_sum(acc[q]);
    if (lane == 0) {
        const int4 p = face_uv[2 * fg], q = face_uv[2 * fg + 1];
        const int64_t du1 = (int64_t)p.z - p.x, dv1 = (int64_t)p.w - p.y;
        const int64_t du2 = (int64_t)q.x - p.x, dv2 = (int64_t)q.y - p.y;
        const int64_t det = du1 * dv2 - du2 * dv1;
        const float sg = det > 0 ? 1.0f : (det < 0 ? -1.0f : 0.0f);
        const float c1 = sg * (float)dv2, c2 = -sg * (float)dv1;
        const float3 tfb = f3(acc[18], acc[19], acc[20]);
        const float3 e1b = mul3(tfb, c1), e2b = mul3(tfb, c2);
        float* o = face_acc + 18 * fg;
        const float3 v0 = sub3(f3(acc[0], acc[1], acc[2]), add3(e1b, e2b));
        const float3 v1 = add3(f3(acc[3], acc[4], acc[5]), e1b);
        const float3 v2 = add3(f3(acc[6], acc[7], acc[8]), e2b);
        st3(o, 0, v0);
        st3(o, 1, v1);
        st3(o, 2, v2);
#pragma unroll
        for (int q2 = 0; q2 < 9; ++q2) o[9 + q2] = acc[9 + q2];
    }
}

__device__ __forceinline__ int corner_of(const int32_t* __restrict__ F, int32_t f, int64_t v) {
    return F[3 * f] == v ? 0 : (F[3 * f + 1] == v ? 1 : 2);
}

// Per low-poly vertex: gather the faces' corner sums (faces ascending), then
// the adjoint of n_v = s_v/|s_v| with s_v recomputed in the forward's order.
__global__ __launch_bounds__(256) void bwd_vertex1_kernel(Batch B, const uint32_t* __restrict__ off,
                                                          const int32_t* __restrict__ adj,
                                                          const float* __restrict__ face_acc_all,
                                                          float* __restrict__ vbar, float* __restrict__ sbar) {
    if (!sealed(B)) return;
    int64_t lb;
    const AssetDev& As = B.A[block_asset(B, kGLoV, blockIdx.x, &lb)];
    const int64_t v = lb * 256 + threadIdx.x;
    if (v >= As.nlv) return;
    const float* V = As.lo_V;
    const int32_t* F = As.lo_F;
    const float* face_acc = face_acc_all + 18 * As.lf;
    const int64_t g = As.lv + v;
    float3 vb = f3(0.f, 0.f, 0.f), nb = f3(0.f, 0.f, 0.f), s = f3(0.f, 0.f, 0.f);
    for (uint32_t i = off[g]; i < off[g + 1]; ++i) {
        const int32_t f = adj[i];
        const int k = corner_of(F, f, v);
        const float* o = face_acc + 18 * (int64_t)f;
        vb = add3(vb, f3(o[3 * k], o[3 * k + 1], o[3 * k + 2]));
        nb = add3(nb, f3(o[9 + 3 * k], o[9 + 3 * k + 1], o[9 + 3 * k + 2]));
        const float3 A = ld3(V, F[3 * f]), Bv = ld3(V, F[3 * f + 1]), C = ld3(V, F[3 * f + 2]);
        const float3 c = cross3(sub3(Bv, A), sub3(C, A));
        s.x += c.x;
        s.y += c.y;
        s.z += c.z;
    }
    const float ls = sqrtf(dot3(s, s));
    float3 sb = f3(0.f, 0.f, 0.f);
    if (ls > 0.f && isfinite(ls)) sb = unit_adj(nb, mul3(s, 1.0f / ls), ls);
    st3(vbar, g, vb);
    st3(sbar, g, sb);
}

// Per low-poly face: c_bar = sum of its vertices' s_bar; adjoint of the cross
// product c = e1 x e2 into corner contributions.
__global__ __launch_bounds__(256) void bwd_face2_kernel(Batch B, const float* __restrict__ sbar_all,
                                                        float* __restrict__ face_acc2) {
    if (!sealed(B)) return;
    int64_t lb;
    const AssetDev& As = B.A[block_asset(B, kGLoF, blockIdx.x, &lb)];
    const int64_t f = lb * 256 + threadIdx.x;
    if (f >= As.nlf) return;
    const float* V = As.lo_V;
    const int32_t* F = As.lo_F;
    const int64_t nv = As.nlv;
    const float* sbar = sbar_all + 3 * As.lv;
    float* o = face_acc2 + 9 * (As.lf + f);
    const int32_t a = F[3 * f], b = F[3 * f + 1], c = F[3 * f + 2];
    if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv) {
        // faces with bad indices never entered the adjacency: nothing to add
        for (int q = 0; q < 9; ++q) o[q] = 0.f;
        return;
    }
    const float3 cb = add3(add3(ld3(sbar, a), ld3(sbar, b)), ld3(sbar, c));
    const float3 A = ld3(V, a), e1 = sub3(ld3(V, b), A), e2 = sub3(ld3(V, c), A);
    const float3 e1b = cross3(e2, cb), e2b = cross3(cb, e1);
    st3(o, 0, mul3(add3(e1b, e2b), -1.0f));
    st3(o, 1, e1b);
    st3(o, 2, e2b);
}

__global__ __launch_bounds__(256) void bwd_vertex2_kernel(Batch B, const uint32_t* __restrict__ off,
                                                          const int32_t* __restrict__ adj,
                                                          const float* __restrict__ face_acc2_all,
                                                          const float* __restrict__ vbar) {
    if (!sealed(B)) return;
    int64_t lb;
    const int ai = block_asset(B, kGLoV, blockIdx.x, &lb);
    const AssetDev& As = B.A[ai];
    float* grad_lo_V = B.G[ai].grad_lo_V;
    const int64_t v = lb * 256 + threadIdx.x;
    if (v >= As.nlv || !grad_lo_V) return;
    const int32_t* F = As.lo_F;
    const float* face_acc2 = face_acc2_all + 9 * As.lf;
    const int64_t g = As.lv + v;
    float3 acc = ld3(vbar, g);
    for (uint32_t i = off[g]; i < off[g + 1]; ++i) {
        const int32_t f = adj[i];
        const int k = corner_of(F, f, v);
        acc = add3(acc, ld3(face_acc2 + 9 * (int64_t)f, k));
    }
    st3(grad_lo_V, v, acc);
}

__global__ __launch_bounds__(256) void zero_grad_hi_kernel(Batch B) {
    if (!sealed(B)) return;
    int64_t lb;
    const int ai = block_asset(B, kGHiV, blockIdx.x, &lb);
    float* out = B.G[ai].grad_hi_N;
    const int64_t v = lb * 256 + threadIdx.x;
    if (!out || v >= B.A[ai].nhv) return;
    st3(out, v, f3(0.f, 0.f, 0.f));
}

// The term of sorted pair j: the hit's barycentric weight of corner k times
// the ray's adjoint of the interpolated high-poly normal (item = 3 ray + k).
__device__ __forceinline__ float3 hiN_term(const uint32_t* __restrict__ vals, const HiTerm* __restrict__ ht,
                                           int64_t j) {
    const uint32_t item = vals[j];
    const uint32_t r = item / 3, k = item - 3 * r;
    const HiTerm h = ht[r];
    const float beta = k == 0 ? 1.0f - h.a.w - h.b.x : (k == 1 ? h.a.w : h.b.x);
    return mul3(f3(h.a.x, h.a.y, h.a.z), beta);
}

// Sorted (vertex, item) pairs of an asset, 64 at a time per wave: each lane
// forms its pair's term, a segmented scan over the wave adds the terms of
// each vertex's run (items ascending within a run: the sort is stable) in a
// fixed tree order, and the lane at the run's end writes the sum.  A run
// that goes on past the wave's 64 pairs is finished by that lane, adding the
// rest in pair order; the waves holding the rest skip it.  Waves take
// (asset, 64-ray batch) items: 192 pairs each.
__global__ __launch_bounds__(256) void bwd_hiN_kernel(Batch B, const uint32_t* __restrict__ keys,
                                                      const uint32_t* __restrict__ vals,
                                                      const HiTerm* __restrict__ ht) {
    if (!sealed(B)) return;
    const int lane = threadIdx.x & 63;
    const uint32_t nb = B.rb_pf[B.n];
    const uint32_t waves = gridDim.x * 4u;
    for (uint32_t q = __builtin_amdgcn_readfirstlane(blockIdx.x * 4u + (threadIdx.x >> 6)); q < nb;
         q += waves) {
        const RayItem it = ray_item(B, q, 0);
        float* grad_hi_N = B.G[it.a].grad_hi_N;
        if (!grad_hi_N) continue;
        const uint32_t nhv = (uint32_t)B.A[it.a].nhv;
        const int64_t lo = 3 * it.begin, hi = 3 * it.end;
        // the three 64-pair groups' loads first (keys, items, then each
        // item's hit and ray gradient), so their latencies overlap; the
        // scans below are unchanged
        uint32_t keyv[3];
        float3 gv[3];
        bool contv[3];
#pragma unroll
        for (int k3 = 0; k3 < 3; ++k3) {
            const int64_t i0 = 3 * it.r + 64 * k3;
            const int64_t i = i0 + lane;
            const bool in = i < hi;  // false for every lane past the batch's pairs
            keyv[k3] = in ? keys[i] : 0xFFFFFFFFu;  // past the end: a run of its own
            gv[k3] = in ? hiN_term(vals, ht, i) : f3(0.f, 0.f, 0.f);
            contv[k3] = i0 < hi && i0 > lo && keys[i0 - 1] == keys[i0];
        }
        for (int k3 = 0; k3 < 3; ++k3) {
            const int64_t i0 = 3 * it.r + 64 * k3;  // the wave's first pair
            if (i0 >= hi) break;
            const int64_t i = i0 + lane;
            const bool in = i < hi;
            const uint32_t key = keyv[k3];
            float3 g = in && key < nhv ? gv[k3] : f3(0.f, 0.f, 0.f);
            const uint32_t prev = __shfl_up(key, 1, 64);
            const uint32_t next = __shfl_down(key, 1, 64);
            bool head = lane == 0 || prev != key;
            // lanes of lane 0's run; it started before this wave when the pair
            // before i0 has the same key
            const uint64_t heads = __ballot(lane > 0 && prev != key);
            const int first_change = heads ? __ffsll((long long)heads) - 1 : 64;
            const bool cont_in = contv[k3];
            // segmented inclusive scan: (v1, f1) then (v2, f2) -> (f2 ? v2 : v1 + v2, f1 | f2)
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const float ux = __shfl_up(g.x, o, 64), uy = __shfl_up(g.y, o, 64), uz = __shfl_up(g.z, o, 64);
                const bool uh = __shfl_up((int)head, o, 64) != 0;
                if (lane >= o) {
                    if (!head) g = f3(ux + g.x, uy + g.y, uz + g.z);
                    head = head || uh;
                }
            }
            const bool run_end = lane == 63 || next != key;
            if (!in || key >= nhv || !run_end) continue;
            if (lane < first_change && cont_in) continue;  // an earlier wave's run
            if (lane == 63) {
                for (int64_t j = i0 + 64; j < hi && keys[j] == key; ++j) g = add3(g, hiN_term(vals, ht, j));
            }
            st3(grad_hi_N, key, g);
        }
    }
}

// Squared-error loss helper: grad = 2 (map - target), per-block partial sums
// of (map - target)^2 over kLossTile values (each thread its values in a fixed
// order), then a single block adds the partials in order.
constexpr int kLossItems = 16;
constexpr int kLossTile = 256 * kLossItems;
__global__ __launch_bounds__(256) void sq_loss_kernel(const float* __restrict__ map,
                                                      const float* __restrict__ target, int64_t n,
                                                      float* __restrict__ grad, float* __restrict__ partial) {
    __shared__ float red[4];
    float e = 0.f;
#pragma unroll 4
    for (int k = 0; k < kLossItems; ++k) {
        const int64_t i = (int64_t)blockIdx.x * kLossTile + (int64_t)k * 256 + threadIdx.x;
        if (i < n) {
            const float d = map[i] - target[i];
            if (grad) grad[i] = 2.0f * d;
            e += d * d;
        }
    }
    e = wave_sum(e);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// The same over 16-byte aligned arrays: each thread loads its 16 values as
// four float4 (one 16-byte access each instead of four 4-byte ones); the last
// block's first n % 4 threads take the values after the last whole float4.
__global__ __launch_bounds__(256) void sq_loss4_kernel(const float4* __restrict__ map,
                                                       const float4* __restrict__ target, int64_t n,
                                                       float4* __restrict__ grad, float* __restrict__ partial) {
    __shared__ float red[4];
    const int64_t n4 = n >> 2;
    float4 m[kLossItems / 4], t[kLossItems / 4];
#pragma unroll
    for (int k = 0; k < kLossItems / 4; ++k) {
        const int64_t i = (int64_t)blockIdx.x * (kLossTile / 4) + (int64_t)k * 256 + threadIdx.x;
        if (i < n4) {
            m[k] = map[i];
            t[k] = target[i];
        }
    }
    float e = 0.f;
#pragma unroll
    for (int k = 0; k < kLossItems / 4; ++k) {
        const int64_t i = (int64_t)blockIdx.x * (kLossTile / 4) + (int64_t)k * 256 + threadIdx.x;
        if (i < n4) {
            const float4 d = make_float4(m[k].x - t[k].x, m[k].y - t[k].y, m[k].z - t[k].z, m[k].w - t[k].w);
            if (grad) grad[i] = make_float4(2.0f * d.x, 2.0f * d.y, 2.0f * d.z, 2.0f * d.w);
            e += d.x * d.x;
            e += d.y * d.y;
            e += d.z * d.z;
            e += d.w * d.w;
        }
    }
    if (blockIdx.x == gridDim.x - 1 && (int64_t)threadIdx.x < n - 4 * n4) {
        const int64_t i = 4 * n4 + threadIdx.x;
        const float d = reinterpret_cast<const float*>(map)[i] - reinterpret_cast<const float*>(target)[i];
        if (grad) reinterpret_cast<float*>(grad)[i] = 2.0f * d;
        e += d * d;
    }
    e = wave_sum(e);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(1024) void sum_partials_kernel(const float* __restrict__ partial, int64_t m,
                                                            float* __restrict__ out) {
    __shared__ float red[16];
    float acc = 0.f;
    for (int64_t i = threadIdx.x; i < m; i += 1024) acc += partial[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int w = 0; w < 16; ++w) s += red[w];
        *out = s;
    }
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_backward(const BatchHost& H, bool any_lo, bool any_hi, hipStream_t s, hipStream_t side,
                           hipEvent_t fork, hipEvent_t join) {
    const Layout& L = H.L;
    char* ws = H.ws;
    hipError_t e;
    const Ray* rays = (const Ray*)(ws + L.rays);
    const Hit* hits = (const Hit*)(ws + L.hits);
    RayGrad* rg = (RayGrad*)(ws + L.bwd_ray);
    HiTerm* ht = (HiTerm*)(ws + L.bwd_hterm);
    // persistent waves over the (asset, 64-ray batch) items: enough for the
    // largest possible ray count, capped
    int64_t cap_batches = 0;
    for (int a = 0; a < L.n; ++a) cap_batches += ((int64_t)H.A[a].res * H.A[a].res + 63) / 64;
    const unsigned ray_grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((cap_batches + 3) / 4, 4096));
    if (L.t_tex > 0) {
        hipLaunchKernelGGL(bwd_ray_kernel, dim3(ray_grid), dim3(256), 0, s, H.dev, rays, hits,
                           (const float4*)(ws + L.lo_n), (const float4*)(ws + L.face_t), rg, ht,
                           (uint32_t*)(ws + L.bwd_k0), (uint32_t*)(ws + L.bwd_v0));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // the low-poly and high-poly gradients only share the per-ray adjoint:
    // with a second stream, the low-poly chain runs beside the sort
    const bool beside = side != nullptr && any_lo && L.t_lv > 0 && any_hi && L.t_hv > 0;
    hipStream_t ls = s;
    bool sorted = false, in1 = false;
    if (beside) {
        // the sort is queued first and the fork recorded after its first
        // histogram: that short latency-bound launch runs alone, the
        // low-poly chain beside the scatters
        if (L.t_tex > 0) {
            if ((e = launch_sort(H, kSortBwd, L.max_hv_bits, &in1, s, fork)) != hipSuccess) return e;
            sorted = true;
        } else if ((e = hipEventRecord(fork, s)) != hipSuccess) {
            return e;
        }
        if ((e = hipStreamWaitEvent(side, fork, 0)) != hipSuccess) return e;
        ls = side;
        // the zeroing of dL/dhi_N goes to the second stream too; the segment
        // sums wait for it (and for the low-poly chain) after the sort
        hipLaunchKernelGGL(zero_grad_hi_kernel, dim3((unsigned)H.blocks(kGHiV)), dim3(256), 0, side, H.dev);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (any_lo && L.t_lv > 0) {
        float* face1 = (float*)(ws + L.bwd_face1);
        float* face2 = (float*)(ws + L.bwd_face2);
        float* sbar = (float*)(ws + L.bwd_sbar);
        float* vbar = (float*)(ws + L.bwd_vbar);
        const uint32_t* off = (const uint32_t*)(ws + L.lo_off);
        const int32_t* adj = (const int32_t*)(ws + L.lo_adj);
        if (H.blocks(kGLoFWave) > 0) {
            hipLaunchKernelGGL(bwd_face_kernel, dim3((unsigned)H.blocks(kGLoFWave)), dim3(256), 0, ls, H.dev,
                               rays, (const RayGrad*)rg, (const uint32_t*)(ws + L.face_off),
                               (const int4*)(ws + L.face_uv), face1);
        }
        hipLaunchKernelGGL(bwd_vertex1_kernel, dim3((unsigned)H.blocks(kGLoV)), dim3(256), 0, ls, H.dev, off,
                           adj, (const float*)face1, vbar, sbar);
        if (H.blocks(kGLoF) > 0) {
            hipLaunchKernelGGL(bwd_face2_kernel, dim3((unsigned)H.blocks(kGLoF)), dim3(256), 0, ls, H.dev,
                               (const float*)sbar, face2);
        }
        hipLaunchKernelGGL(bwd_vertex2_kernel, dim3((unsigned)H.blocks(kGLoV)), dim3(256), 0, ls, H.dev, off,
                           adj, (const float*)face2, (const float*)vbar);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (beside && (e = hipEventRecord(join, side)) != hipSuccess) return e;
    if (any_hi && L.t_hv > 0) {
        if (!beside) {
            hipLaunchKernelGGL(zero_grad_hi_kernel, dim3((unsigned)H.blocks(kGHiV)), dim3(256), 0, s, H.dev);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        if (L.t_tex > 0) {
            if (!sorted && (e = launch_sort(H, kSortBwd, L.max_hv_bits, &in1, s)) != hipSuccess) return e;
            if (beside && (e = hipStreamWaitEvent(s, join, 0)) != hipSuccess) return e;
            hipLaunchKernelGGL(bwd_hiN_kernel, dim3(ray_grid), dim3(256), 0, s, H.dev,
                               (const uint32_t*)(ws + (in1 ? L.bwd_k1 : L.bwd_k0)),
                               (const uint32_t*)(ws + (in1 ? L.bwd_v1 : L.bwd_v0)), (const HiTerm*)ht);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    if (beside && (e = hipStreamWaitEvent(s, join, 0)) != hipSuccess) return e;
    return hipSuccess;
}

hipError_t launch_sq_loss(const float* map, const float* target, int64_t n3, float* grad, float* loss,
                          float* partial, hipStream_t s) {
    if (n3 <= 0) return fill_u32((uint32_t*)loss, 0u, 1, s);
    const unsigned nb = blocks_for(n3, kLossTile);
    if ((((uintptr_t)map | (uintptr_t)target | (uintptr_t)grad) & 15) == 0)
        hipLaunchKernelGGL(sq_loss4_kernel, dim3(nb), dim3(256), 0, s, (const float4*)map, (const float4*)target, n3,
                           (float4*)grad, partial);
    else
        hipLaunchKernelGGL(sq_loss_kernel, dim3(nb), dim3(256), 0, s, map, target, n3, grad, partial);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(1024), 0, s, (const float*)partial, (int64_t)nb, loss);
    return hipGetLastError();
}

}  // namespace bake
