// Per-texel correspondence query and tangent-space encoding (Sec. 6.4): for
// each covered texel, build the ray from the G-buffer (world position and
// interpolated smooth normal), find the high-poly hit with the smallest |t| in
// [-max_dist, +max_dist] (ties to the lower original triangle index),
// interpolate the high-poly normal with the hit's barycentric weights and
// project it into the texel's tangent frame.
//
// Traversal (two launch shapes, same per-ray arithmetic and results):
//   * wave batches (default): persistent waves take (asset, 64-ray batch)
//     items of the batch's face-ordered ray lists from device work queues
//     (one per XCD, each over a contiguous eighth of the items first: see
//     next_item), trace the 64 rays together in a tight loop and encode when the whole
//     batch is done: neighbouring texels of one face walk nearly the same
//     nodes, and the asset is uniform across the wave.  The loop's trips are
//     all-internal-node or all-leaf, a leaf trip being taken once at least
//     half of the busy lanes wait at a leaf (the balanced loop), or phased,
//     or mixed (see traverse_batch_kernel);
//   * lane refill: lanes whose ray finished are refilled from a ray queue over
//     the concatenated lists while the rest continue (wave-level compaction
//     after Aila & Laine 2009); lanes may then work on different assets;
//   * conservative slab test on the compressed node itself: a child plane is
//     o + q s (frame origin o, power-of-two step s, byte q), so its crossing
//     is t = q (s/d) + (o - p)/d, one fma per plane from three per-node
//     products, with the near / far bytes of both children picked by a byte
//     permute whose selector follows the signs of d.  The slabs are widened
//     outward by an absolute per-ray margin that bounds the FP32 rounding of
//     that evaluation (the error analysis, after Ize 2013, is at make_rayt);
//     a zero direction component takes 1/d = 2^64 instead of infinity, which
//     the margin turns into an unbounded slab for a ray inside it and a
//     rejected box for a ray outside;
//   * hit rule: a triangle is hit when the crossing's barycentric weights are
//     all >= -kEdgeEps (relative edge tolerance) and |t| <= max_dist; the
//     winner minimises (floor(|t| / w), index) with the quantum w = max_dist
//     2^-20, so a ray through a shared edge or vertex, or two surfaces at the
//     same distance, resolve to the lower index instead of to rounding noise;
//   * pruning keeps every node whose nearest |t| reaches the best key's bin,
//     so the result equals a brute-force scan under the same triangle test,
//     independent of the tree and of the visiting order;
//   * watertight ray/triangle test (Woop, Benthin & Wald 2013): shear to ray
//     space, edge functions as differences of two rounded products with FP
//     contraction off, so a shared edge gives exactly opposite values in the
//     two faces; two-sided;
//   * short per-lane stack in LDS, spilling its oldest entries to a per-lane
//     global area when full (the Karras tree depth is bounded by 62).
// The closest-point query (the paper's own form) shares the traversal: boxes
// are pruned by their distance from the texel position, triangles report the
// distance of their nearest point, and the same (distance bin, index) rule
// picks the winner.
#include <algorithm>

#include "internal.h"

namespace bake {

namespace {

constexpr int32_t kEmpty = INT32_MIN;
constexpr float kPad = 1e-6f;
constexpr float kEdgeEps = 1.0f / 16384.0f;   // must match the leaf-box widening in lbvh.hip
constexpr float kQuantScale = 1048576.0f;    // 2^20: distance quantum w = max_dist / 2^20
constexpr uint32_t kFaceReliable = 1u;

struct float3x3 {
    float3 r0, r1, r2;
};

__device__ __forceinline__ float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return f3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float3 ld3(const float* p, int64_t i) {
    return f3(p[3 * i], p[3 * i + 1], p[3 * i + 2]);
}
__device__ __forceinline__ float comp(float3 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

// Edge function of two sheared vertices, as a difference of two rounded
// products (no FMA): swapping the arguments negates the result exactly.
__device__ __forceinline__ float edge_fn(float xa, float ya, float xb, float yb) {
#pragma clang fp contract(off)
    float p = xa * yb;
    float q = ya * xb;
    return p - q;
}

// Ray state for the slab and triangle tests.
struct RayT {
    float3 p;
    float3 invd;    // 1/d, magnitudes clamped to 2^64 (2^64 for a zero component)
    float3 E;       // per-axis slab margin, in units of t
    uint32_t seln;  // byte-permute selector of the left child's near planes
    float3x3 S;     // rows of the shear: (Ax, Ay, Az) = S (v - p)
};

constexpr float kInvdMax = 18446744073709551616.0f;  // 2^64
constexpr float kSlabRel = 1.0f / 1048576.0f;        // 2^-20

// The slab margin.  A compressed child plane is the exact value o + q s,
// which the build places on the outer side of the child's box up to half an
// ulp of the coordinate (it checks the once-rounded fmaf(q, s, o)); the test
// evaluates t = fma(q, A, B) with A = s c exact (c the stored 1/d, s a power
// of two), B = fl(fl(o - p) c -+ E).  With u = 2^-24, X = the largest
// coordinate magnitude of the root box and M1 = the largest distance from p
// to it (every frame origin and plane lies in the root box, 255 s is at most
// twice the node's extent), the errors are at most 2uX|c| (plane), uM1|c|
// (o - p), u(M1|c| + E) (B), and, where a slab end can decide the test (|t|
// within about twice the bound b <= max_dist), 2ub for the final rounding and
// 2ub for c against 1/d: in all below E / 4 with E = 2^-20 ((M1 + X)|c| +
// max_dist).  In space that widens every box by about 1e-6 of (scene extent +
// coordinate magnitude).  A clamped c (|d| < 2^-64) scales the slab ends
// towards zero, but only for planes within E / |c| of p, which the margin
// already makes unbounded.  A non-finite root frame gives a NaN margin: every
// slab is then unbounded (the NaN-ignoring min3 / max3).
__device__ __forceinline__ RayT make_rayt(float3 p, float3 d, const BvhNodeC* root, float max_dist) {
    RayT r;
    r.p = p;
    auto inv = [](float x) {
        const float c = x == 0.f ? kInvdMax : 1.0f / x;
        return fabsf(c) > kInvdMax ? copysignf(kInvdMax, c) : c;
    };
    r.invd = f3(inv(d.x), inv(d.y), inv(d.z));
    // near byte of the left child per axis: lo (bytes 0, 1, 2) for d >= 0,
    // hi (bytes 3, 4, 5) for d < 0; byte 3 of the selector yields zero
    r.seln = (d.x < 0.f ? 3u : 0u) | ((d.y < 0.f ? 4u : 1u) << 8) | ((d.z < 0.f ? 5u : 2u) << 16) | (0x0Cu << 24);
    r.E = f3(0.f, 0.f, 0.f);
    if (root) {
        const float4 a = root->a;
        const uint32_t meta = __float_as_uint(a.w);
        auto margin = [&](float o, uint32_t e, float pc, float c) {
            const float hi = fmaf(255.f, __uint_as_float(e << 23), o);
            const float m1 = fmaxf(fabsf(o - pc), fabsf(hi - pc)), x = fmaxf(fabsf(o), fabsf(hi));
            return kSlabRel * fmaf(m1 + x, fabsf(c), max_dist);
        };
        r.E = f3(margin(a.x, meta & 0xFFu, p.x, r.invd.x), margin(a.y, (meta >> 8) & 0xFFu, p.y, r.invd.y),
                 margin(a.z, (meta >> 16) & 0xFFu, p.z, r.invd.z));
    }
    float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    int kz = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    if (comp(d, kz) < 0.f) {
        int t = kx; kx = ky; ky = t;
    }
    float dz = comp(d, kz);
    float Sx = comp(d, kx) / dz, Sy = comp(d, ky) / dz, Sz = 1.0f / dz;
    float rx[3] = {0.f, 0.f, 0.f}, ry[3] = {0.f, 0.f, 0.f}, rz[3] = {0.f, 0.f, 0.f};
    rx[kx] = 1.f; rx[kz] = -Sx;
    ry[ky] = 1.f; ry[kz] = -Sy;
    rz[kz] = Sz;
    r.S.r0 = f3(rx[0], rx[1], rx[2]);
    r.S.r1 = f3(ry[0], ry[1], ry[2]);
    r.S.r2 = f3(rz[0], rz[1], rz[2]);
    return r;
}

__device__ __forceinline__ float3 shear(const RayT& r, float3 v) {
    float3 a = f3(v.x - r.p.x, v.y - r.p.y, v.z - r.p.z);
    return f3(fmaf(r.S.r0.z, a.z, fmaf(r.S.r0.y, a.y, r.S.r0.x * a.x)),
              fmaf(r.S.r1.z, a.z, fmaf(r.S.r1.y, a.y, r.S.r1.x * a.x)),
              fmaf(r.S.r2.z, a.z, fmaf(r.S.r2.y, a.y, r.S.r2.x * a.x)));
}

struct Best {
    uint32_t key;   // floor(|t| / w), 0xFFFFFFFF before the first hit
    int32_t id;     // INT32_MAX before the first hit
    float t, b1, b2;
    float bound;    // prune nodes whose nearest |t| exceeds this
};

// Watertight test, two-sided (|t| <= max_dist) or ONE-sided (0 < t <=
// max_dist); on a better (key, id) hit updates the best.
template <bool ONE = false>
__device__ __forceinline__ void tri_test(const RayT& r, const Leaf& L, float max_dist, float inv_w,
                                         float w, Best* b) {
    float3 v0 = f3(L.a.x, L.a.y, L.a.z), v1 = f3(L.a.w, L.b.x, L.b.y), v2 = f3(L.b.z, L.b.w, L.c.x);
    int32_t id = __float_as_int(L.c.y);
    float3 A = shear(r, v0), B = shear(r, v1), C = shear(r, v2);
    float U = edge_fn(C.x, C.y, B.x, B.y);
    float V = edge_fn(A.x, A.y, C.x, C.y);
    float W = edge_fn(B.x, B.y, A.x, A.y);
    float det = U + V + W;
    // written without branches (the lanes of a leaf trip take one path; a
    // zero det gives a non-finite t, which the range test rejects)
    const bool neg = det < 0.f;
    U = neg ? -U : U;
    V = neg ? -V : V;
    W = neg ? -W : W;
    det = neg ? -det : det;
    const bool inside = det != 0.f && !(fminf(fminf(U, V), W) < -kEdgeEps * det);
    // T accumulated in this order, each product fused into the next sum
    const float T = fmaf(W, C.z, fmaf(V, B.z, U * A.z));
    float rdet = 1.0f / det;
    float t = T * rdet;
    float at = fabsf(t);
    const bool in_range = ONE ? (t > 0.f && t <= max_dist) : (at <= max_dist);
    const uint32_t key = in_range ? (uint32_t)(at * inv_w) : 0xFFFFFFFFu;
    const bool better = inside && in_range && (key < b->key || (key == b->key && id < b->id));
    b->key = better ? key : b->key;
    b->id = better ? id : b->id;
    b->t = better ? t : b->t;
    b->b1 = better ? V * rdet : b->b1;
    b->b2 = better ? W * rdet : b->b2;
    b->bound = better ? (float)(key + 1u) * w * (1.0f + kPad) : b->bound;
}

// Point-to-box distance test: true when the box may hold a point within
// `bound` of p; *d2 = the squared distance (0 inside).  The FP32 rounding of
// d2 is a few 2^-24 relative, well inside the bound's 1e-6 pad.
__device__ __forceinline__ bool box_dist_test(float3 p, float3 lo, float3 hi, float bound, float* d2) {
    const float dx = fmaxf(fmaxf(lo.x - p.x, p.x - hi.x), 0.f);
    const float dy = fmaxf(fmaxf(lo.y - p.y, p.y - hi.y), 0.f);
    const float dz = fmaxf(fmaxf(lo.z - p.z, p.z - hi.z), 0.f);
    *d2 = dx * dx + dy * dy + dz * dz;
    return *d2 <= bound * bound;
}

__device__ __forceinline__ bool coord_less(float3 a, float3 b) {
    return a.x < b.x || (a.x == b.x && (a.y < b.y || (a.y == b.y && a.z < b.z)));
}

// Nearest point of a leaf triangle to p: the orthogonal projection when its
// barycentric weights are all >= 0, else the nearest of the edges' nearest
// points.  On a better (distance bin, index) updates the best, with t = the
// distance and (b1, b2) = the weights of corners 1 and 2.
__device__ __forceinline__ void tri_closest_test(float3 p, const Leaf& L, float max_dist, float inv_w,
                                                 float w, Best* b) {
    const float3 v[3] = {f3(L.a.x, L.a.y, L.a.z), f3(L.a.w, L.b.x, L.b.y), f3(L.b.z, L.b.w, L.c.x)};
    const int32_t id = __float_as_int(L.c.y);
    const float3 e1 = f3(v[1].x - v[0].x, v[1].y - v[0].y, v[1].z - v[0].z);
    const float3 e2 = f3(v[2].x - v[0].x, v[2].y - v[0].y, v[2].z - v[0].z);
    const float3 n = cross3(e1, e2);
    const float nn = dot3(n, n);
    float dist = INFINITY, w1 = 0.f, w2 = 0.f;
    bool inside = false;
    if (nn > 0.f) {
        const float3 ap = f3(p.x - v[0].x, p.y - v[0].y, p.z - v[0].z);
        const float sd = dot3(n, ap);
        const float k = sd / nn;
        const float3 q = f3(p.x - k * n.x, p.y - k * n.y, p.z - k * n.z);
        const float inv = 1.0f / nn;
        const float3 q0 = f3(v[0].x - q.x, v[0].y - q.y, v[0].z - q.z);
        const float3 q1 = f3(v[1].x - q.x, v[1].y - q.y, v[1].z - q.z);
        const float3 q2 = f3(v[2].x - q.x, v[2].y - q.y, v[2].z - q.z);
        const float wa = dot3(n, cross3(q1, q2)) * inv;
        const float wb = dot3(n, cross3(q2, q0)) * inv;
        const float wc = dot3(n, cross3(q0, q1)) * inv;
        if (wa >= 0.f && wb >= 0.f && wc >= 0.f) {
            inside = true;
            dist = fabsf(sd) / sqrtf(nn);
            w1 = wb;
            w2 = wc;
        }
    }
    if (!inside) {
        // an edge's distance is computed from its endpoints in a fixed
        // (coordinate) order, and an endpoint's as |p - v|, so triangles that
        // share the edge or vertex get bitwise the same value and a closest
        // point there resolves to the lower index
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            int i = e, j = e == 2 ? 0 : e + 1;
            if (coord_less(v[j], v[i])) {
                const int t = i; i = j; j = t;
            }
            const float3 u = v[i];
            const float3 ab = f3(v[j].x - u.x, v[j].y - u.y, v[j].z - u.z);
            const float3 up = f3(p.x - u.x, p.y - u.y, p.z - u.z);
            const float l2 = dot3(ab, ab);
            float s = l2 > 0.f ? dot3(up, ab) / l2 : 0.f;
            float de;
            if (s <= 0.f) {
                s = 0.f;
                de = sqrtf(dot3(up, up));
            } else if (s >= 1.f) {
                s = 1.f;
                const float3 vp = f3(p.x - v[j].x, p.y - v[j].y, p.z - v[j].z);
                de = sqrtf(dot3(vp, vp));
            } else {
                const float3 r = f3(up.x - s * ab.x, up.y - s * ab.y, up.z - s * ab.z);
                de = sqrtf(dot3(r, r));
            }
            if (de < dist) {
                dist = de;
                // weights of corners 1 and 2 for the point u + s (v_j - u)
                w1 = (i == 1 ? 1.f - s : 0.f) + (j == 1 ? s : 0.f);
                w2 = (i == 2 ? 1.f - s : 0.f) + (j == 2 ? s : 0.f);
            }
        }
    }
    if (!(dist <= max_dist)) return;
    const uint32_t key = (uint32_t)(dist * inv_w);
    if (key < b->key || (key == b->key && id < b->id)) {
        b->key = key;
        b->id = id;
        b->t = dist;
        b->b1 = w1;
        b->b2 = w2;
        b->bound = (float)(key + 1u) * w * (1.0f + kPad);
    }
}

struct TravArgs {
    Batch B;
    const Ray* rays;       // concatenated face-ordered ray lists
    const float4* lo_n;    // concatenated lo vertex normals
    const float4* face_t;  // concatenated per-face tangents
    const int4* face_uv;   // concatenated snapped UVs + flags
    const BvhNodeC* nodes;  // concatenated trees
    const Leaf* leaves;
    Hit* hits;             // optional, by global ray index
    int32_t* spill;        // [kMaxDepth][spill_lanes]
    int64_t spill_lanes;
    int32_t xcd_split;     // wave batches: per-XCD work queues (next_item)
};

// What the inner loop needs of an asset.
struct TreeView {
    const BvhNodeC* nodes;
    const Leaf* leaves;
    float max_dist, w, inv_w;
    int32_t root;      // root ref, or kEmpty when there is no triangle
    int32_t step_cap;  // per-ray safety bound on loop steps
};

__device__ __forceinline__ TreeView tree_view(const TravArgs& t, const AssetDev& As) {
    TreeView v;
    v.nodes = t.nodes + As.node;
    v.leaves = t.leaves + As.hf;
    v.max_dist = As.max_dist;
    v.w = As.max_dist / kQuantScale;  // exact: power-of-two scaling
    v.inv_w = kQuantScale / As.max_dist;
    v.root = As.nhf <= 0 ? kEmpty : (As.nhf == 1 ? ~0 : 0);
    v.step_cap = (int32_t)min((int64_t)4 * As.nhf + 1024, (int64_t)INT32_MAX);
    return v;
}

// Node `node` (>= 0) and leaf ~node (node < 0) of a tree.
__device__ __forceinline__ const BvhNodeC* node_at(const TreeView& tv, int32_t node) { return tv.nodes + node; }
__device__ __forceinline__ const Leaf* leaf_at(const TreeView& tv, int32_t node) { return tv.leaves + ~node; }

// Ray setup from the G-buffer record: world position p, interpolated smooth
// normal d, tangent T' orthogonalised against d, UV handedness.  rel = false
// when the face or the frame is degenerate (the texel is unreliable).
struct RaySetup {
    float3 p, d, Tp;
    float hsign;
    int32_t texel;
    bool rel;
};

__device__ __forceinline__ RaySetup setup_ray(const TravArgs& a, const AssetDev& As, const Ray& ray) {
    RaySetup r;
    r.texel = ray.texel;
    const int32_t face = ray.face;
    const float4* lo_n = a.lo_n + As.lv;
    float b1 = ray.b1, b2 = ray.b2, b0 = 1.0f - b1 - b2;
    int32_t i0 = As.lo_F[3 * face], i1 = As.lo_F[3 * face + 1], i2 = As.lo_F[3 * face + 2];
    float3 V0 = ld3(As.lo_V, i0), V1 = ld3(As.lo_V, i1), V2 = ld3(As.lo_V, i2);
    float4 n0 = lo_n[i0], n1 = lo_n[i1], n2 = lo_n[i2];
    r.p = f3(b0 * V0.x + b1 * V1.x + b2 * V2.x, b0 * V0.y + b1 * V1.y + b2 * V2.y,
             b0 * V0.z + b1 * V1.z + b2 * V2.z);
    float3 m = f3(b0 * n0.x + b1 * n1.x + b2 * n2.x, b0 * n0.y + b1 * n1.y + b2 * n2.y,
                  b0 * n0.z + b1 * n1.z + b2 * n2.z);
    const int64_t fg = As.lf + face;
    float4 T4 = a.face_t[fg];
    uint32_t fl = (uint32_t)a.face_uv[2 * fg + 1].z;
    bool rel = (fl & kFaceReliable) && n0.w != 0.f && n1.w != 0.f && n2.w != 0.f;
    float l2 = dot3(m, m);
    rel = rel && l2 > 0.f;
    float rl = rel ? 1.0f / sqrtf(l2) : 0.f;
    r.d = f3(m.x * rl, m.y * rl, m.z * rl);
    float3 T = f3(T4.x, T4.y, T4.z);
    float dt = dot3(r.d, T);
    float3 Tp = f3(T.x - dt * r.d.x, T.y - dt * r.d.y, T.z - dt * r.d.z);
    float lt2 = dot3(Tp, Tp);
    rel = rel && lt2 > 0.f;
    float rt = rel ? 1.0f / sqrtf(lt2) : 0.f;
    r.Tp = f3(Tp.x * rt, Tp.y * rt, Tp.z * rt);
    r.hsign = T4.w;
    r.rel = rel;
    return r;
}

// Interpolate the hit's high-poly normal, project it into (T', B', d) and
// write the texel; unreliable and missed rays get (0,0,1).
__device__ __forceinline__ void finish_ray(const TravArgs& a, const AssetDev& As, int64_t ridx,
                                           const RaySetup& rs, const Best& best) {
    float3 out = f3(0.f, 0.f, 1.f);
    int32_t st = rs.rel ? kMiss : kUnreliable;
    float beta1 = 0.f, beta2 = 0.f, tt = 0.f;
    if (rs.rel && best.id != INT32_MAX) {
        int32_t g = best.id;
        const int32_t* hi_F = As.hi_F;
        const int64_t nhv = As.nhv;
        int32_t j0 = hi_F[3 * (int64_t)g], j1 = hi_F[3 * (int64_t)g + 1], j2 = hi_F[3 * (int64_t)g + 2];
        bool ok = j0 >= 0 && j1 >= 0 && j2 >= 0 && j0 < nhv && j1 < nhv && j2 < nhv;
        beta1 = best.b1;
        beta2 = best.b2;
        tt = best.t;
        float beta0 = 1.0f - beta1 - beta2;
        st = kUnreliable;
        if (ok) {
            float3 N0 = ld3(As.hi_N, j0), N1 = ld3(As.hi_N, j1), N2 = ld3(As.hi_N, j2);
            float3 h = f3(beta0 * N0.x + beta1 * N1.x + beta2 * N2.x,
                          beta0 * N0.y + beta1 * N1.y + beta2 * N2.y,
                          beta0 * N0.z + beta1 * N1.z + beta2 * N2.z);
            float lh2 = dot3(h, h);
            if (lh2 > 0.f && isfinite(lh2)) {
                float rh = 1.0f / sqrtf(lh2);
                float3 n = f3(h.x * rh, h.y * rh, h.z * rh);
                float3 c = cross3(rs.d, rs.Tp);
                float3 Bp = f3(rs.hsign * c.x, rs.hsign * c.y, rs.hsign * c.z);
                out = f3(dot3(n, rs.Tp), dot3(n, Bp), dot3(n, rs.d));
                st = g;
            }
        }
    }
    const int64_t t = rs.texel;
    As.out_map[3 * t] = out.x;
    As.out_map[3 * t + 1] = out.y;
    As.out_map[3 * t + 2] = out.z;
    As.out_hit[t] = st;
    if (a.hits) {
        Hit h;
        h.t = tt;
        h.beta1 = beta1;
        h.beta2 = beta2;
        h.id = st;
        a.hits[ridx] = h;
    }
}

// Per-lane short stack: entries [lo, sp) in LDS (ring of STACK), older ones
// spilled to a per-lane column of global memory.
template <int BLOCK, int STACK>
struct LaneStack {
    int32_t (*lds)[BLOCK];
    int32_t* spill;
    int64_t stride, col;
    int sp, lo;

    __device__ __forceinline__ void push(int32_t x, int tid, uint32_t* status) {
        if (sp - lo == STACK) {
            // the tree depth bound keeps lo < kMaxDepth; the check only
            // guards against a malformed tree
            if (lo < kMaxDepth) spill[(int64_t)lo * stride + col] = lds[lo & (STACK - 1)][tid];
            else atomicOr(status, kStInternal);
            ++lo;
        }
        lds[sp & (STACK - 1)][tid] = x;
        ++sp;
    }
    __device__ __forceinline__ int32_t pop(int tid) {
        if (sp == 0) return kEmpty;
        --sp;
        if (sp < lo) {
            lo = sp;
            return lo < kMaxDepth ? spill[(int64_t)lo * stride + col] : kEmpty;
        }
        return lds[sp & (STACK - 1)][tid];
    }
};

// The child boxes and references of a compressed node (two 16-B loads).
struct NodeBoxes {
    float3 llo, lhi, rlo, rhi;
    int32_t left, right;
};

__device__ __forceinline__ float byte_f(uint32_t w, int k) { return (float)((w >> (8 * k)) & 0xFFu); }

__device__ __forceinline__ NodeBoxes load_node(const BvhNodeC* nd) {
    const float4 a = nd->a;
    const uint4 q = nd->q;
    const uint32_t meta = __float_as_uint(a.w);
    const float sx = __uint_as_float((meta & 0xFFu) << 23), sy = __uint_as_float(((meta >> 8) & 0xFFu) << 23),
                sz = __uint_as_float(((meta >> 16) & 0xFFu) << 23);
    NodeBoxes n;
    n.llo = f3(fmaf(byte_f(q.x, 0), sx, a.x), fmaf(byte_f(q.x, 1), sy, a.y), fmaf(byte_f(q.x, 2), sz, a.z));
    n.lhi = f3(fmaf(byte_f(q.x, 3), sx, a.x), fmaf(byte_f(q.y, 0), sy, a.y), fmaf(byte_f(q.y, 1), sz, a.z));
    n.rlo = f3(fmaf(byte_f(q.y, 2), sx, a.x), fmaf(byte_f(q.y, 3), sy, a.y), fmaf(byte_f(q.z, 0), sz, a.z));
    n.rhi = f3(fmaf(byte_f(q.z, 1), sx, a.x), fmaf(byte_f(q.z, 2), sy, a.y), fmaf(byte_f(q.z, 3), sz, a.z));
    const int32_t g = (int32_t)(q.w & kChildIndex);
    n.left = (q.w & kChildLeafL) ? ~g : g;
    n.right = (q.w & kChildLeafR) ? ~(g + 1) : g + 1;
    return n;
}

// Slab test of one child from its near and far plane bytes (bytes 0-2 of the
// permuted words, x y z): on overlap of the widened slabs with [-bound, bound]
// (ONE: with [0, bound], the half-line) returns true and the smallest |t| of
// the overlap in *mint.
template <bool ONE>
__device__ __forceinline__ bool child_test(uint32_t nw, uint32_t fw, float3 A, float3 Bn, float3 Bf, float bound,
                                           float* mint) {
    const float t0x = fmaf((float)(nw & 0xFFu), A.x, Bn.x), t1x = fmaf((float)(fw & 0xFFu), A.x, Bf.x);
    const float t0y = fmaf((float)((nw >> 8) & 0xFFu), A.y, Bn.y), t1y = fmaf((float)((fw >> 8) & 0xFFu), A.y, Bf.y);
    const float t0z = fmaf((float)((nw >> 16) & 0xFFu), A.z, Bn.z),
                t1z = fmaf((float)((fw >> 16) & 0xFFu), A.z, Bf.z);
    const float t0 = fmaxf(fmaxf(fmaxf(t0x, t0y), t0z), ONE ? 0.f : -bound);
    const float t1 = fminf(fminf(fminf(t1x, t1y), t1z), bound);
    *mint = fmaxf(fmaxf(t0, -t1), 0.f);  // nearest |t| of [t0, t1]
    return t0 <= t1;
}

// One traversal step of a lane at an internal node: test both child boxes, go
// to the nearer hit and push the other, or pop when neither is hit.  Returns
// the next node (internal, leaf, or kEmpty: the ray is done).
template <int BLOCK, int STACK, bool COUNT, bool ONE = false>
__device__ __forceinline__ int32_t inner_step(const TreeView& tv, uint32_t* status, int32_t node,
                                              const RayT& R, const Best& best, LaneStack<BLOCK, STACK>& st,
                                              int tid, unsigned long long& c_box) {
    const BvhNodeC* nd = node_at(tv, node);
    const float4 a = nd->a;
    const uint4 q = nd->q;
    const uint32_t meta = __float_as_uint(a.w);
    // per axis: A = s / d (exact), Bn / Bf = (o - p) / d -/+ the margin
    const float3 A = f3(__uint_as_float((meta & 0xFFu) << 23) * R.invd.x,
                        __uint_as_float(((meta >> 8) & 0xFFu) << 23) * R.invd.y,
                        __uint_as_float(((meta >> 16) & 0xFFu) << 23) * R.invd.z);
    const float dx = a.x - R.p.x, dy = a.y - R.p.y, dz = a.z - R.p.z;
    const float3 Bn = f3(fmaf(dx, R.invd.x, -R.E.x), fmaf(dy, R.invd.y, -R.E.y), fmaf(dz, R.invd.z, -R.E.z));
    const float3 Bf = f3(fmaf(dx, R.invd.x, R.E.x), fmaf(dy, R.invd.y, R.E.y), fmaf(dz, R.invd.z, R.E.z));
    // plane bytes: left child = bytes 0-5 of (q.x, q.y), right = bytes 2-7 of
    // (q.y, q.z); far selector = near with lo / hi swapped per axis
    const uint32_t selF = R.seln ^ 0x00070503u;
    const uint32_t nL = __builtin_amdgcn_perm(q.y, q.x, R.seln), fL = __builtin_amdgcn_perm(q.y, q.x, selF);
    const uint32_t nR = __builtin_amdgcn_perm(q.z, q.y, R.seln + 0x00020202u),
                   fR = __builtin_amdgcn_perm(q.z, q.y, selF + 0x00020202u);
    const int32_t g = (int32_t)(q.w & kChildIndex);
    const int4 ref = make_int4((q.w & kChildLeafL) ? ~g : g, (q.w & kChildLeafR) ? ~(g + 1) : g + 1, 0, 0);
    float mL, mR;
    bool hL = child_test<ONE>(nL, fL, A, Bn, Bf, best.bound, &mL);
    bool hR = child_test<ONE>(nR, fR, A, Bn, Bf, best.bound, &mR);
    if (COUNT) c_box += 2;
    int32_t next = kEmpty;
    if (hL && hR) {
        bool rfirst = mR < mL;
        next = rfirst ? ref.y : ref.x;
        st.push(rfirst ? ref.x : ref.y, tid, status);
    } else if (hL) {
        next = ref.x;
    } else if (hR) {
        next = ref.y;
    }
    if (next == kEmpty) next = st.pop(tid);
    return next;
}

// A lane at a leaf: triangle test, then pop.
template <int BLOCK, int STACK, bool COUNT, bool ONE = false>
__device__ __forceinline__ int32_t leaf_step(const TreeView& tv, int32_t node, const RayT& R, Best& best,
                                             LaneStack<BLOCK, STACK>& st, int tid, unsigned long long& c_tri) {
    const Leaf L = *leaf_at(tv, node);
    tri_test<ONE>(R, L, tv.max_dist, tv.inv_w, tv.w, &best);
    if (COUNT) c_tri += 1;
    return st.pop(tid);
}

// The same two steps for the closest-point query (p = the texel position).
template <int BLOCK, int STACK, bool COUNT>
__device__ __forceinline__ int32_t inner_step_pt(const TreeView& tv, uint32_t* status, int32_t node,
                                                 float3 p, const Best& best, LaneStack<BLOCK, STACK>& st,
                                                 int tid, unsigned long long& c_box) {
    const NodeBoxes nb = load_node(node_at(tv, node));
    const int4 ref = make_int4(nb.left, nb.right, 0, 0);
    float dL, dR;
    bool hL = box_dist_test(p, nb.llo, nb.lhi, best.bound, &dL);
    bool hR = box_dist_test(p, nb.rlo, nb.rhi, best.bound, &dR);
    if (COUNT) c_box += 2;
    int32_t next = kEmpty;
    if (hL && hR) {
        bool rfirst = dR < dL;
        next = rfirst ? ref.y : ref.x;
        st.push(rfirst ? ref.x : ref.y, tid, status);
    } else if (hL) {
        next = ref.x;
    } else if (hR) {
        next = ref.y;
    }
    if (next == kEmpty) next = st.pop(tid);
    return next;
}

template <int BLOCK, int STACK, bool COUNT>
__device__ __forceinline__ int32_t leaf_step_pt(const TreeView& tv, int32_t node, float3 p, Best& best,
                                                LaneStack<BLOCK, STACK>& st, int tid, unsigned long long& c_tri) {
    const Leaf L = *leaf_at(tv, node);
    tri_closest_test(p, L, tv.max_dist, tv.inv_w, tv.w, &best);
    if (COUNT) c_tri += 1;
    return st.pop(tid);
}

// One step of either kind.
template <int BLOCK, int STACK, bool COUNT>
__device__ __forceinline__ int32_t trav_step(const TreeView& tv, uint32_t* status, int32_t node,
                                             const RayT& R, Best& best, LaneStack<BLOCK, STACK>& st,
                                             int tid, unsigned long long& c_box, unsigned long long& c_tri) {
    if (node >= 0) return inner_step<BLOCK, STACK, COUNT>(tv, status, node, R, best, st, tid, c_box);
    return leaf_step<BLOCK, STACK, COUNT>(tv, node, R, best, st, tid, c_tri);
}

__device__ __forceinline__ void reset_best(Best& b, float max_dist) {
    b.key = 0xFFFFFFFFu;
    b.id = INT32_MAX;
    b.t = b.b1 = b.b2 = 0.f;
    b.bound = max_dist * (1.0f + kPad);
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Query kinds of the shared traversal: the two-sided ray of the bake, the
// closest point (p = R.p), the first hit of a half-line (camera rays).
constexpr int kQRay = 0, kQPoint = 1, kQFirst = 2;

// One internal-node or leaf step of a query.
template <int BLOCK, int STACK, bool COUNT, int Q>
__device__ __forceinline__ int32_t node_step(const TreeView& tv, uint32_t* status, int32_t node,
                                             const RayT& R, Best& best, LaneStack<BLOCK, STACK>& st, int tid,
                                             unsigned long long& c_box) {
    if constexpr (Q == kQPoint) return inner_step_pt<BLOCK, STACK, COUNT>(tv, status, node, R.p, best, st, tid, c_box);
    else return inner_step<BLOCK, STACK, COUNT, Q == kQFirst>(tv, status, node, R, best, st, tid, c_box);
}
template <int BLOCK, int STACK, bool COUNT, int Q>
__device__ __forceinline__ int32_t tri_step(const TreeView& tv, int32_t node, const RayT& R, Best& best,
                                            LaneStack<BLOCK, STACK>& st, int tid, unsigned long long& c_tri) {
    if constexpr (Q == kQPoint) return leaf_step_pt<BLOCK, STACK, COUNT>(tv, node, R.p, best, st, tid, c_tri);
    else return leaf_step<BLOCK, STACK, COUNT, Q == kQFirst>(tv, node, R, best, st, tid, c_tri);
}

// The XCD (0..7) whose compute unit runs the calling wave, from the hardware
// register that names it.
__device__ __forceinline__ int wave_xcd() {
    return (int)(__builtin_amdgcn_s_getreg((3 << 11) | 20) & (kXcds - 1));  // hwreg(HW_REG_XCC_ID, 0, 4)
}

// The work queue of the wave batches: the wave's next (asset, 64-ray batch)
// item of the n in face order, n when none is left.  With one queue every
// wave takes the next item, so the waves in flight (about 7,000 on 256 CUs)
// cover a window of about 40 % of a 1M-ray bake, spread over all eight XCDs.
// With the XCD split the items are cut into kXcds contiguous ranges and a
// wave takes from its own XCD's range first: the waves that share an L2 then
// trace one region of the surface, whose nodes and leaves stay in that L2.
// A wave whose range is done moves on to the next XCD's range (cur, left: the
// range it takes from and how many ranges it has yet to find empty); a range
// once found empty stays empty, so every wave ends after at most kXcds
// empty answers and every item is handed out exactly once.
struct ItemQueue {
    int cur, left;
};

__device__ __forceinline__ ItemQueue item_queue_init(bool split) {
    ItemQueue iq;
    iq.cur = split ? wave_xcd() : 0;
    iq.left = split ? kXcds : 1;
    return iq;
}

__device__ __forceinline__ uint32_t next_item(const Batch& B, uint32_t n, bool split, int lane, ItemQueue& iq) {
    for (;;) {
        if (iq.left == 0) return n;
        uint32_t lo = 0, len = n;
        uint32_t* head = &B.gcnt[kGcQueue];
        if (split) {
            lo = (uint32_t)(((uint64_t)n * (uint32_t)iq.cur) / kXcds);
            len = (uint32_t)(((uint64_t)n * (uint32_t)(iq.cur + 1)) / kXcds) - lo;
            head = &B.gcnt[kGcXcdQueue + kXcdStride * iq.cur];
        }
        uint32_t k = 0;
        if (lane == 0) k = atomicAdd(head, 1u);
        k = __builtin_amdgcn_readfirstlane(__shfl(k, 0, 64));
        if (k < len) return lo + k;
        --iq.left;
        iq.cur = iq.cur + 1 == kXcds ? 0 : iq.cur + 1;
    }
}

// Loop shapes of the wave batches (TravConfig::mode):
constexpr int kLoopSingle = 0;    // every trip: each lane one step of its own kind
constexpr int kLoopPhased = 2;    // internal-node trips until every lane is at a leaf, then one leaf trip
constexpr int kLoopBalanced = 3;  // each trip is all-leaf or all-internal: a leaf trip once at least
                                  // half of the busy lanes wait at a leaf

// Wave batches: each wave takes one (asset, 64-ray batch) item at a time,
// traces its rays together and encodes once all 64 are done.  Each lane's
// sequence of steps is the same under every loop shape (it depends only on
// its ray and the tree); the shapes differ in how the wave interleaves its
// lanes' internal-node and leaf steps.  A trip that mixes both kinds costs
// the wave both code paths; the phased shape (after Aila & Laine's
// while-while loop) never mixes them but makes lanes that reached a leaf
// early wait through the rest of the internal-node phase; the balanced shape
// never mixes them and lets no more than half of the busy lanes wait.
template <int BLOCK, int STACK, bool COUNT, int LOOP, bool CLOSEST>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(COUNT ? 1 : 7))) void traverse_batch_kernel(TravArgs a) {
    __shared__ int32_t stk[STACK][BLOCK];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const Batch& B = a.B;
    const uint32_t nbatches = B.rb_pf[B.n];
    LaneStack<BLOCK, STACK> st;
    st.lds = stk;
    st.spill = a.spill;
    st.stride = a.spill_lanes;
    st.col = (int64_t)blockIdx.x * BLOCK + tid;
    const bool split = a.xcd_split != 0;
    ItemQueue iq = item_queue_init(split);
    for (;;) {
        const uint32_t q = next_item(B, nbatches, split, lane, iq);
        if (q >= nbatches) break;
        const int ai = upper_asset(B.rb_pf, B.n, q);
        const AssetDev& As = B.A[ai];
        const TreeView tv = tree_view(a, As);
        const uint32_t nr = B.cnt[(int64_t)ai * kCntSlots + kCntRays];
        const uint32_t k = (q - B.rb_pf[ai]) * 64u + (uint32_t)lane;  // asset-local ray
        const int64_t r = (int64_t)B.ray_pf[ai] + k;                    // global ray
        int32_t node = kEmpty;
        Best best;
        reset_best(best, tv.max_dist);
        RayT R;
        if (k < nr) {
            // the setup is recomputed for the encode below, so it is not
            // kept live through the traversal loop
            const RaySetup rs = setup_ray(a, As, a.rays[r]);
            if (rs.rel) {
                if constexpr (CLOSEST) R.p = rs.p;
                else R = make_rayt(rs.p, rs.d, tv.root >= 0 ? tv.nodes : nullptr, tv.max_dist);
                node = tv.root;
            }
        }
        st.sp = st.lo = 0;
        int32_t steps = 0;
        unsigned long long c_box = 0, c_tri = 0, c_iter = 0;  // c_iter: trips of the whole wave
        // a lane past the step bound (only a malformed tree gets there) stops
        auto capped = [&]() {
            if (++steps > tv.step_cap) {
                set_status(B, kStInternal);
                node = kEmpty;
            }
        };
        if constexpr (LOOP == kLoopPhased) {
            while (__ballot(node != kEmpty)) {
                while (__ballot(node >= 0)) {
                    if (COUNT) ++c_iter;
                    if (node >= 0) {
                        node = node_step<BLOCK, STACK, COUNT, CLOSEST ? kQPoint : kQRay>(tv, B.status, node, R, best, st, tid, c_box);
                        capped();
                    }
                }
                if (COUNT && __ballot(node != kEmpty)) ++c_iter;
                if (node != kEmpty) {
                    node = tri_step<BLOCK, STACK, COUNT, CLOSEST ? kQPoint : kQRay>(tv, node, R, best, st, tid, c_tri);
                    capped();
                }
            }
        } else if constexpr (LOOP == kLoopBalanced) {
            // internal-node trips while more busy lanes are at an internal
            // node than at a leaf, then one leaf trip; the node trips leave
            // the best hit untouched, so their loop keeps it in place
            for (;;) {
                uint64_t at_leaf;
                for (;;) {
                    const uint64_t at_node = __ballot(node >= 0);
                    at_leaf = __ballot(node < 0 && node != kEmpty);
                    if (__popcll(at_leaf) >= __popcll(at_node)) break;
                    if (COUNT) ++c_iter;
                    if (node >= 0) {
                        node = node_step<BLOCK, STACK, COUNT, CLOSEST ? kQPoint : kQRay>(tv, B.status, node, R, best, st, tid, c_box);
                        capped();
                    }
                }
                if (at_leaf == 0) break;  // and no lane at a node: the batch is done
                if (COUNT) ++c_iter;
                if (node < 0 && node != kEmpty) {
                    node = tri_step<BLOCK, STACK, COUNT, CLOSEST ? kQPoint : kQRay>(tv, node, R, best, st, tid, c_tri);
                    capped();
                }
            }
        } else {
            while (__ballot(node != kEmpty)) {
                if (COUNT) ++c_iter;
                if (node >= 0) {
                    node = node_step<BLOCK, STACK, COUNT, CLOSEST ? kQPoint : kQRay>(tv, B.status, node, R, best, st, tid, c_box);
                    capped();
                } else if (node != kEmpty) {
                    node = tri_step<BLOCK, STACK, COUNT, CLOSEST ? kQPoint : kQRay>(tv, node, R, best, st, tid, c_tri);
                    capped();
                }
            }
        }
        if (k < nr) finish_ray(a, As, r, setup_ray(a, As, a.rays[r]), best);
        if (COUNT) {
            c_box = wave_sum_u64(c_box);
            c_tri = wave_sum_u64(c_tri);
            if (lane == 0) {
                atomicAdd((unsigned long long*)&B.cnt[(int64_t)ai * kCntSlots + kCntBoxLo], c_box);
                atomicAdd((unsigned long long*)&B.cnt[(int64_t)ai * kCntSlots + kCntTriLo], c_tri);
                atomicAdd((unsigned long long*)&B.cnt[(int64_t)ai * kCntSlots + kCntIterLo], c_iter);
            }
        }
    }
}

// Camera rays of the hidden-face pass (Sec. 6.2): view v is a pinhole at
// eye_v looking at the target; forward f, helper a = the world axis with the
// smallest |target_k - eye_k| (lowest k on ties), right r = normalise(f x a),
// up u = r x f; pixel (i, j) of
// the res x res image looks along normalise(f + x r + y u) with x = ((j +
// 1/2) 2 / res - 1) tan_half and y = (1 - (i + 1/2) 2 / res) tan_half.  Each
// wave takes an 8 x 8 pixel tile of one view (grid-stride over the (view,
// tile) items; lanes past the image edge idle), so its 64 rays leave the eye
// in a square bundle and walk similar paths, finds every ray's first hit on
// the half-line (0, t_far] with the bake's hit rule and flags the hit face
// visible.
struct VisArgs {
    TravArgs t;
    const float* eyes;
    float3 target;
    float tan_half;
    int32_t n_views, res;
    uint32_t* visible;   // NULL: no visibility flags
    int32_t* first_hit;  // NULL or per pixel
    float* depth;        // NULL or per pixel: distance t of the first hit along the ray, +inf for none
};

// The pinhole frame of a view (forward, right, up; see visibility_kernel).
// The helper axis is chosen on the exact FP64 differences target - eye, so
// the choice is the same however the forward vector rounds.
__device__ __forceinline__ void view_frame(float3 e, float3 target, float3* f_out, float3* r_out, float3* u_out) {
    const double ax = fabs((double)target.x - (double)e.x), ay = fabs((double)target.y - (double)e.y),
                 az = fabs((double)target.z - (double)e.z);
    float3 f = f3(target.x - e.x, target.y - e.y, target.z - e.z);
    const float rf = 1.0f / sqrtf(dot3(f, f));
    f = f3(f.x * rf, f.y * rf, f.z * rf);
    int k = 0;
    if (ay < ax) k = 1;
    if (az < (k == 0 ? ax : ay)) k = 2;
    float3 r = cross3(f, f3(k == 0 ? 1.f : 0.f, k == 1 ? 1.f : 0.f, k == 2 ? 1.f : 0.f));
    const float rr = 1.0f / sqrtf(dot3(r, r));
    r = f3(r.x * rr, r.y * rr, r.z * rr);
    *f_out = f;
    *r_out = r;
    *u_out = cross3(r, f);
}

// Eye, unit direction and view forward of pixel p of view v.
__device__ __forceinline__ void pixel_ray(const VisArgs& a, int32_t v, int64_t p, float3* e_out, float3* d_out,
                                          float3* f_out) {
    const float3 e = ld3(a.eyes, v);
    float3 f, r, u;
    view_frame(e, a.target, &f, &r, &u);
    const int32_t i = (int32_t)(p / a.res), j = (int32_t)(p - (int64_t)i * a.res);
    const float x = (((float)j + 0.5f) * 2.0f / (float)a.res - 1.0f) * a.tan_half;
    const float y = (1.0f - ((float)i + 0.5f) * 2.0f / (float)a.res) * a.tan_half;
    float3 d = f3(f.x + x * r.x + y * u.x, f.y + x * r.y + y * u.y, f.z + x * r.z + y * u.z);
    const float rd = 1.0f / sqrtf(dot3(d, d));
    *e_out = e;
    *d_out = f3(d.x * rd, d.y * rd, d.z * rd);
    *f_out = f;
}

template <int BLOCK, int STACK, bool COUNT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(COUNT ? 1 : 7))) void visibility_kernel(VisArgs a) {
    __shared__ int32_t stk[STACK][BLOCK];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const Batch& B = a.t.B;
    const TreeView tv = tree_view(a.t, B.A[0]);
    LaneStack<BLOCK, STACK> st;
    st.lds = stk;
    st.spill = a.t.spill;
    st.stride = a.t.spill_lanes;
    st.col = (int64_t)blockIdx.x * BLOCK + tid;
    const int64_t px = (int64_t)a.res * a.res;
    const int64_t tpr = ((int64_t)a.res + 7) / 8;  // 8 x 8 tiles per image row
    const int64_t tpv = tpr * tpr;                 // tiles per view
    const int64_t items = tpv * a.n_views;
    const int64_t nwaves = ((int64_t)gridDim.x * BLOCK) >> 6;
    unsigned long long c_box = 0, c_tri = 0, c_iter = 0;
    for (int64_t it = ((int64_t)blockIdx.x * BLOCK + tid) >> 6; it < items; it += nwaves) {
        const int32_t v = (int32_t)(it / tpv);
        const int64_t t = it - (int64_t)v * tpv, ty = t / tpr, tx = t - ty * tpr;
        const int64_t row = ty * 8 + (lane >> 3), col = tx * 8 + (lane & 7);
        const bool valid = row < a.res && col < a.res;
        const int64_t p = valid ? row * a.res + col : 0;
        RayT R;
        {
            float3 e, d, f;
            pixel_ray(a, v, p, &e, &d, &f);
            R = make_rayt(e, d, tv.root >= 0 ? tv.nodes : nullptr, tv.max_dist);
        }
        int32_t node = valid ? tv.root : kEmpty;
        Best best;
        reset_best(best, tv.max_dist);
        st.sp = st.lo = 0;
        int32_t steps = 0;
        // a lane past the step bound (only a malformed tree gets there) stops
        auto capped = [&]() {
            if (++steps > tv.step_cap) {
                set_status(B, kStInternal);
                node = kEmpty;
            }
        };
        // the balanced loop as nested loops, as in the bake's wave batches:
        // internal-node trips while more busy lanes are at an internal node
        // than at a leaf, then one leaf trip
        for (;;) {
            uint64_t at_leaf;
            for (;;) {
                const uint64_t at_node = __ballot(node >= 0);
                at_leaf = __ballot(node < 0 && node != kEmpty);
                if (__popcll(at_leaf) >= __popcll(at_node)) break;
                if (COUNT) ++c_iter;
                if (node >= 0) {
                    node = node_step<BLOCK, STACK, COUNT, kQFirst>(tv, B.status, node, R, best, st, tid, c_box);
                    capped();
                }
            }
            if (at_leaf == 0) break;  // and no lane at a node: the tile is done
            if (COUNT) ++c_iter;
            if (node < 0 && node != kEmpty) {
                node = tri_step<BLOCK, STACK, COUNT, kQFirst>(tv, node, R, best, st, tid, c_tri);
                capped();
            }
        }
        if (valid) {
            const int32_t id = best.id == INT32_MAX ? -1 : best.id;
            if (a.first_hit) a.first_hit[(int64_t)v * px + p] = id;
            if (a.depth) a.depth[(int64_t)v * px + p] = id >= 0 ? best.t : INFINITY;
            if (id >= 0 && a.visible) a.visible[id] = 1u;
        }
    }
    if (COUNT) {
        c_box = wave_sum_u64(c_box);
        c_tri = wave_sum_u64(c_tri);
        if (lane == 0) {
            atomicAdd((unsigned long long*)&B.cnt[kCntBoxLo], c_box);
            atomicAdd((unsigned long long*)&B.cnt[kCntTriLo], c_tri);
            atomicAdd((unsigned long long*)&B.cnt[kCntIterLo], c_iter);
        }
    }
}

// Backprojection precompute (Sec. 7.4, TextureGen Postprocessing): per covered texel of asset 0 (its
// surface point p and smooth normal from the G-buffer) and per view: image
// coordinates col = (q.r / (z tan_half) + 1) res / 2 - 1/2, row = (1 - q.u /
// (z tan_half)) res / 2 - 1/2 with q = p - e, z = q.f (pixel centres at
// integers; (-1, -1) outside the image or behind the eye), and the incidence
// max(0, n . (e - p) / |e - p|), set to 0 when z exceeds the depth buffer at
// the nearest pixel by more than tol (occluded) or the normal is undefined.
struct MapArgs {
    TravArgs t;
    const float* eyes;
    float3 target;
    float tan_half;
    int32_t n_views, img_res;
    const float* depth;  // [n_views][img_res^2] first-hit distances along the pixel rays
    float tol;
    float* uv_out;       // [n_views][res^2][2]
    float* inc_out;      // [n_views][res^2]
};

__global__ __launch_bounds__(256) void view_map_kernel(MapArgs a) {
    const Batch& B = a.t.B;
    const AssetDev& As = B.A[0];
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= (int64_t)B.cnt[kCntRays]) return;
    const Ray ray = a.t.rays[r];
    const float b1 = ray.b1, b2 = ray.b2, b0 = 1.0f - b1 - b2;
    const int32_t i0 = As.lo_F[3 * ray.face], i1 = As.lo_F[3 * ray.face + 1], i2 = As.lo_F[3 * ray.face + 2];
    const float3 V0 = ld3(As.lo_V, i0), V1 = ld3(As.lo_V, i1), V2 = ld3(As.lo_V, i2);
    const float4 n0 = a.t.lo_n[i0], n1 = a.t.lo_n[i1], n2 = a.t.lo_n[i2];
    const float3 p = f3(b0 * V0.x + b1 * V1.x + b2 * V2.x, b0 * V0.y + b1 * V1.y + b2 * V2.y,
                        b0 * V0.z + b1 * V1.z + b2 * V2.z);
    float3 n = f3(b0 * n0.x + b1 * n1.x + b2 * n2.x, b0 * n0.y + b1 * n1.y + b2 * n2.y,
                  b0 * n0.z + b1 * n1.z + b2 * n2.z);
    const float l2 = dot3(n, n);
    const bool ok = l2 > 0.f;
    const float rl = ok ? 1.0f / sqrtf(l2) : 0.f;
    n = f3(n.x * rl, n.y * rl, n.z * rl);
    const int64_t texels = (int64_t)As.res * As.res, tex = ray.texel;
    const int64_t px = (int64_t)a.img_res * a.img_res;
    const float half = 0.5f * (float)a.img_res;
    for (int32_t k = 0; k < a.n_views; ++k) {
        const float3 e = ld3(a.eyes, k);
        float3 f, rt, u;
        view_frame(e, a.target, &f, &rt, &u);
        const float3 q = f3(p.x - e.x, p.y - e.y, p.z - e.z);
        const float z = dot3(q, f);
        float col = -1.f, row = -1.f, inc = 0.f;
        if (z > 0.f) {
            const float c = (dot3(q, rt) / (z * a.tan_half) + 1.0f) * half - 0.5f;
            const float w = (1.0f - dot3(q, u) / (z * a.tan_half)) * half - 0.5f;
            const float hi = (float)a.img_res - 0.5f;
            if (c >= -0.5f && c < hi && w >= -0.5f && w < hi) {
                col = c;
                row = w;
                if (ok) {
                    const int32_t pi = min(max((int32_t)floorf(w + 0.5f), 0), a.img_res - 1);
                    const int32_t pj = min(max((int32_t)floorf(c + 0.5f), 0), a.img_res - 1);
                    // the pixel ray's hit distance to view-axis depth: d . f =
                    // 1 / |f + x r + y u| = 1 / sqrt(1 + x^2 + y^2)
                    const float x = (((float)pj + 0.5f) / half - 1.0f) * a.tan_half;
                    const float y = (1.0f - ((float)pi + 0.5f) / half) * a.tan_half;
                    const float zb = a.depth[(int64_t)k * px + (int64_t)pi * a.img_res + pj] / sqrtf(1.0f + x * x + y * y);
                    if (!(z > zb + a.tol)) {
                        const float3 dk = f3(-q.x, -q.y, -q.z);
                        const float cs = dot3(n, dk) / sqrtf(dot3(dk, dk));
                        inc = fmaxf(cs, 0.f);
                    }
                }
            }
        }
        a.uv_out[2 * ((int64_t)k * texels + tex)] = col;
        a.uv_out[2 * ((int64_t)k * texels + tex) + 1] = row;
        a.inc_out[(int64_t)k * texels + tex] = inc;
    }
}

// Lane refill: idle lanes take new rays from the ray queue when at least 16
// of the wave are idle; the rest keep traversing.  Each lane finds the asset
// of its ray.
template <int BLOCK, int STACK, bool COUNT>
__global__ __launch_bounds__(BLOCK) void traverse_refill_kernel(TravArgs a) {
    __shared__ int32_t stk[STACK][BLOCK];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const Batch& B = a.B;
    const uint32_t nrays = B.ray_pf[B.n];
    LaneStack<BLOCK, STACK> st;
    st.lds = stk;
    st.spill = a.spill;
    st.stride = a.spill_lanes;
    st.col = (int64_t)blockIdx.x * BLOCK + tid;
    st.sp = st.lo = 0;
    bool active = false, exhausted = false;
    uint32_t ridx = 0;
    int ai = 0;
    RaySetup rs;
    rs.rel = false;
    RayT R;
    Best best;
    TreeView tv = tree_view(a, B.A[0]);
    reset_best(best, tv.max_dist);
    int32_t node = kEmpty;
    int32_t steps = 0;
    // c_iter: trips of the whole wave, kept by the lowest active lane (so a
    // trip is attributed to that lane's asset)
    unsigned long long c_box = 0, c_tri = 0, c_iter = 0;
    for (;;) {
        uint64_t idle = __ballot(!active);
        if (!exhausted && (int)__popcll(idle) >= 16) {
            int cnt = (int)__popcll(idle);
            int leader = __ffsll((long long)idle) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(&B.gcnt[kGcQueue], (uint32_t)cnt);
            base = __shfl(base, leader, 64);
            if (base >= nrays) exhausted = true;
            if (!active) {
                uint32_t k = base + (uint32_t)__popcll(idle & __lanemask_lt());
                if (k < nrays) {
                    if (COUNT && (c_box | c_tri | c_iter)) {
                        atomicAdd((unsigned long long*)&B.cnt[(int64_t)ai * kCntSlots + kCntBoxLo], c_box);
                        atomicAdd((unsigned long long*)&B.cnt[(int64_t)ai * kCntSlots + kCntTriLo], c_tri);
                        atomicAdd((unsigned long long*)&B.cnt[(int64_t)ai * kCntSlots + kCntIterLo], c_iter);
                        c_box = c_tri = c_iter = 0;
                    }
                    ridx = k;
                    ai = upper_asset(B.ray_pf, B.n, k);
                    const AssetDev& As = B.A[ai];
                    tv = tree_view(a, As);
                    rs = setup_ray(a, As, a.rays[k]);
                    reset_best(best, tv.max_dist);
                    node = rs.rel ? tv.root : kEmpty;
                    st.sp = st.lo = 0;
                    steps = 0;
                    if (rs.rel) R = make_rayt(rs.p, rs.d, tv.root >= 0 ? tv.nodes : nullptr, tv.max_dist);
                    active = node != kEmpty;
                    if (!active) finish_ray(a, As, k, rs, best);
                }
            }
        }
        if (__ballot(active) == 0) {
            if (exhausted) break;
            continue;
        }
        if (!active) continue;
        if (COUNT && (__ballot(true) & __lanemask_lt()) == 0) ++c_iter;
        node = trav_step<BLOCK, STACK, COUNT>(tv, B.status, node, R, best, st, tid, c_box, c_tri);
        if (++steps > tv.step_cap) {
            set_status(B, kStInternal);
            node = kEmpty;
        }
        if (node != kEmpty) continue;
        active = false;
        finish_ray(a, B.A[ai], ridx, rs, best);
    }
    if (COUNT && (c_box | c_tri | c_iter)) {
        atomicAdd((unsigned long long*)&B.cnt[(int64_t)ai * kCntSlots + kCntBoxLo], c_box);
        atomicAdd((unsigned long long*)&B.cnt[(int64_t)ai * kCntSlots + kCntTriLo], c_tri);
        atomicAdd((unsigned long long*)&B.cnt[(int64_t)ai * kCntSlots + kCntIterLo], c_iter);
    }
}

// MODE: TravConfig::mode (the closest-point query has no lane-refill kernel:
// mode 1 runs the balanced loop there).
template <int BLOCK, int STACK, bool COUNT, int MODE, bool CLOSEST>
hipError_t launch_one(const TravArgs& args, hipStream_t s, int64_t max_lanes) {
    static int cached_blocks = -1;
    auto kern = (MODE == 1 && !CLOSEST) ? traverse_refill_kernel<BLOCK, STACK, COUNT>
                                        : traverse_batch_kernel<BLOCK, STACK, COUNT, MODE == 1 ? kLoopBalanced : MODE,
                                                                CLOSEST>;
    if (cached_blocks < 0) {
        int dev = 0, cus = 0, per = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, BLOCK, 0);
        if (e != hipSuccess) return e;
        if (per < 1) per = 1;
        cached_blocks = cus * per;
    }
    int64_t blocks = cached_blocks;
    int64_t cap = max_lanes / BLOCK;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(BLOCK), 0, s, args);
    return hipGetLastError();
}

template <int BLOCK, int STACK, bool COUNT, bool CLOSEST>
hipError_t launch_mode_q(const TravArgs& args, int mode, hipStream_t s, int64_t max_lanes) {
    switch (mode) {
        case 0: return launch_one<BLOCK, STACK, COUNT, 0, CLOSEST>(args, s, max_lanes);
        case 1: return launch_one<BLOCK, STACK, COUNT, 1, CLOSEST>(args, s, max_lanes);
        case 2: return launch_one<BLOCK, STACK, COUNT, 2, CLOSEST>(args, s, max_lanes);
        case 3: return launch_one<BLOCK, STACK, COUNT, 3, CLOSEST>(args, s, max_lanes);
    }
    return hipErrorInvalidValue;
}

template <int BLOCK, int STACK, bool COUNT>
hipError_t launch_mode(const TravArgs& args, int mode, bool closest, hipStream_t s, int64_t max_lanes) {
    if (closest) return launch_mode_q<BLOCK, STACK, COUNT, true>(args, mode, s, max_lanes);
    return launch_mode_q<BLOCK, STACK, COUNT, false>(args, mode, s, max_lanes);
}

}  // namespace

hipError_t launch_visibility_rays(const BatchHost& H, const VisRun& v, hipStream_t s) {
    const Layout& L = H.L;
    char* ws = H.ws;
    if (v.n_views <= 0 || v.res <= 0) return hipSuccess;
    constexpr int kBlk = 256, kStk = 16;
    VisArgs a;
    a.t.B = H.dev;
    a.t.rays = nullptr;
    a.t.lo_n = nullptr;
    a.t.face_t = nullptr;
    a.t.face_uv = nullptr;
    a.t.nodes = (const BvhNodeC*)(ws + L.nodes_c);
    a.t.leaves = (const Leaf*)(ws + L.leaves);
    a.t.hits = nullptr;
    a.t.spill = v.spill;
    a.t.spill_lanes = v.spill_lanes;
    a.t.xcd_split = 0;
    a.eyes = v.eyes;
    a.target = make_float3(v.target[0], v.target[1], v.target[2]);
    a.tan_half = v.tan_half;
    a.n_views = v.n_views;
    a.res = v.res;
    a.visible = v.visible;
    a.first_hit = v.first_hit;
    a.depth = v.depth;
    auto kern = v.count ? visibility_kernel<kBlk, kStk, true> : visibility_kernel<kBlk, kStk, false>;
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kBlk, 0)) != hipSuccess) return e;
    const int64_t tpr = ((int64_t)v.res + 7) / 8;
    const int64_t waves = tpr * tpr * v.n_views;  // one 8 x 8 pixel tile per wave item
    int64_t blocks = (int64_t)cus * std::max(per, 1);
    blocks = std::min(blocks, (waves + kBlk / 64 - 1) / (kBlk / 64));  // no block without an item
    blocks = std::min(blocks, v.spill_lanes / kBlk);                    // every lane has a spill column
    blocks = std::max<int64_t>(blocks, 1);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kBlk), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_view_maps(const BatchHost& H, const MapRun& m, hipStream_t s) {
    const Layout& L = H.L;
    char* ws = H.ws;
    if (L.t_tex == 0 || m.n_views <= 0) return hipSuccess;
    MapArgs a;
    a.t.B = H.dev;
    a.t.rays = (const Ray*)(ws + L.rays);
    a.t.lo_n = (const float4*)(ws + L.lo_n);
    a.t.face_t = nullptr;
    a.t.face_uv = nullptr;
    a.t.nodes = nullptr;
    a.t.leaves = nullptr;
    a.t.hits = nullptr;
    a.t.spill = nullptr;
    a.t.spill_lanes = 0;
    a.t.xcd_split = 0;
    a.eyes = m.eyes;
    a.target = make_float3(m.target[0], m.target[1], m.target[2]);
    a.tan_half = m.tan_half;
    a.n_views = m.n_views;
    a.img_res = m.img_res;
    a.depth = m.depth;
    a.tol = m.tol;
    a.uv_out = m.uv_out;
    a.inc_out = m.inc_out;
    // one thread per texel of the atlas bounds the covered texels (rays)
    const unsigned blocks = (unsigned)((L.t_tex + 255) / 256);
    hipLaunchKernelGGL(view_map_kernel, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_traverse(const BatchHost& H, const TravConfig& cfg, hipStream_t s) {
    const Layout& L = H.L;
    char* ws = H.ws;
    // the queue heads (the single queue and the per-XCD ones) start at zero:
    // the forward zeroes every counter before its first launch, and the
    // traversal is its only user of them
    if (L.t_tex == 0) return hipSuccess;
    TravArgs a;
    a.B = H.dev;
    a.rays = (const Ray*)(ws + L.rays);
    a.lo_n = (const float4*)(ws + L.lo_n);
    a.face_t = (const float4*)(ws + L.face_t);
    a.face_uv = (const int4*)(ws + L.face_uv);
    a.nodes = (const BvhNodeC*)(ws + L.nodes_c);
    a.leaves = (const Leaf*)(ws + L.leaves);
    a.hits = L.save ? (Hit*)(ws + L.hits) : nullptr;
    a.spill = (int32_t*)(ws + L.spill);
    a.spill_lanes = L.spill_lanes;
    a.xcd_split = cfg.xcd ? 1 : 0;
    int64_t lanes = L.spill_lanes;
    if (cfg.count) return launch_mode<256, 16, true>(a, cfg.mode, cfg.closest, s, lanes);
#define BAKE_TRAV_CASE(B, S) \
    if (cfg.block == B && cfg.stack == S) return launch_mode<B, S, false>(a, cfg.mode, cfg.closest, s, lanes);
    BAKE_TRAV_CASE(64, 8) BAKE_TRAV_CASE(64, 16) BAKE_TRAV_CASE(64, 32)
    BAKE_TRAV_CASE(128, 8) BAKE_TRAV_CASE(128, 16) BAKE_TRAV_CASE(128, 32)
    BAKE_TRAV_CASE(256, 8) BAKE_TRAV_CASE(256, 16) BAKE_TRAV_CASE(256, 32)
#undef BAKE_TRAV_CASE
    return hipErrorInvalidValue;
}

}  // namespace bake
