// Internal declarations of the gfx950 normal baker: record layouts shared by
// the kernels and the launchers called by the C ABI layer (api.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bake {

// ---------------------------------------------------------------------------
// Records
// ---------------------------------------------------------------------------

// One covered texel: the ray list is in face order (faces ascending, texels of a
// face in row-major order of its UV bounding box) so neighbouring lanes trace
// neighbouring rays.
struct Ray {
    int32_t texel;
    int32_t face;
    float b1, b2;  // barycentrics of lo corners 1 and 2; b0 = 1 - b1 - b2
};
static_assert(sizeof(Ray) == 16, "Ray is 16 B");

// Result of the correspondence query, saved for the backward pass.
struct Hit {
    float t;
    float beta1, beta2;  // weights of hi corners 1 and 2; beta0 = 1 - beta1 - beta2
    int32_t id;          // hi triangle (original index), or a negative status
};
static_assert(sizeof(Hit) == 16, "Hit is 16 B");

// Binary BVH node holding the boxes of both children (64 B, one cache line
// fetch per visit):
//   a = (L.lo.x, L.lo.y, L.lo.z, L.hi.x)
//   b = (L.hi.y, L.hi.z, R.lo.x, R.lo.y)
//   c = (R.lo.z, R.hi.x, R.hi.y, R.hi.z)
//   ref = (left, right, -, -): >= 0 internal node, < 0 leaf ~ref
struct alignas(16) BvhNode {
    float4 a, b, c;
    int4 ref;
};
static_assert(sizeof(BvhNode) == 64, "BvhNode is 64 B");

// Leaf triangle: vertices copied from hi_V (bit-exact) plus original index.
//   a = (v0.x, v0.y, v0.z, v1.x), b = (v1.y, v1.z, v2.x, v2.y),
//   c = (v2.z, id as bits, -, -)
struct alignas(16) Leaf {
    float4 a, b, c;
};
static_assert(sizeof(Leaf) == 48, "Leaf is 48 B");

// Maximum stack depth a traversal can need.  In the Karras hierarchy the
// common-prefix length strictly grows from parent to child and lies in
// [2, 63] for 30-bit keys extended by the 32-bit index, so a root-to-leaf
// path has at most 62 internal nodes.
constexpr int kMaxDepth = 64;

// Device status word bits (mirror of BAKE_STATUS_* in bake.h).
constexpr uint32_t kStLoIndex = 1u, kStHiIndex = 2u, kStBadUV = 4u, kStNonFinite = 8u,
                   kStInternal = 16u;

// Per-ray status values (mirror of bake.h).
constexpr int32_t kMiss = -1, kUnreliable = -2, kUncovered = -3;

// ---------------------------------------------------------------------------
// Workspace layout (byte offsets into the caller's workspace)
// ---------------------------------------------------------------------------
struct Layout {
    size_t status, counters;                 // u32 status word; counters (see kCnt*)
    size_t lo_n, lo_deg, lo_off, lo_cur, lo_adj;  // lo vertex normals + vertex->face CSR
    size_t face_t, face_uv, face_cnt, face_off;   // per lo face
    size_t scan_tmp;                          // block sums for the scans
    size_t facemap, level;                    // per texel
    size_t rays, hits;                        // per ray
    size_t bounds_part, bounds;               // centroid bounds reduction
    size_t keys0, keys1, vals0, vals1, hist;  // radix sort
    size_t nodes, leaves, node_parent, leaf_parent, refit_cnt, node_range, frontier, treelets;
    size_t spill;                             // traversal stack spill
    // backward scratch (BAKE_FLAG_SAVE only)
    size_t bwd_ray, bwd_k0, bwd_v0, bwd_k1, bwd_v1, bwd_hist, bwd_face1, bwd_face2, bwd_sbar, bwd_vbar;
    size_t total;
    // sizes used by launchers
    int64_t n_texels, max_rays, sort_blocks, scan_tmp_n, spill_lanes;
};

// counters[] slots
constexpr int kCntRays = 0;      // number of covered texels (rays)
constexpr int kCntQueue = 1;     // persistent traversal work queue head
constexpr int kCntBoxLo = 2;     // u64 box tests (FLAG_COUNT), slots 2-3
constexpr int kCntTriLo = 4;     // u64 triangle tests (FLAG_COUNT), slots 4-5
constexpr int kCntFrontier = 6;  // refit frontier length
constexpr int kCntTreelets = 7;  // number of refit treelets

// Capacity of the treelet list and of the refit frontier.  Treelet roots are
// the small children of the nodes with more than 2048 leaves ("big" nodes).
// Big nodes whose children are both small cover disjoint ranges of > 2048
// leaves, so there are fewer than n / 2048 of them, and every big node lies
// on the root path (at most 62 nodes) of one of them: fewer than 62 n / 2048
// + 62 big nodes, one more treelet than big nodes.
inline int64_t treelet_cap(int64_t n) { return n / 32 + 2 * kMaxDepth + 16; }
constexpr int kCntSlots = 16;

// Traversal configuration
struct TravConfig {
    int block;    // 64 / 128 / 256
    int stack;    // LDS entries per lane: 8 / 16 / 32
    int persist;  // 1: refill finished lanes from a work queue; 0: static striding
    bool count = false;  // instrumented variant: count box and triangle tests
};

// ---------------------------------------------------------------------------
// Launchers (all asynchronous on `s`)
// ---------------------------------------------------------------------------
hipError_t fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s);

// Exclusive scan of n u32 values; writes out[0..n) and, if total != nullptr,
// the sum to *total (device).  tmp needs scan_tmp_elems(n) u32.
int64_t scan_tmp_elems(int64_t n);
hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp,
                              uint32_t* total, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on the low `bits` bits, 8 per
// pass, ping-ponging between (k0, v0) and (k1, v1); *result_in_1 tells where
// the sorted pairs ended.  hist needs radix_hist_elems(n) u32.  With n_dev the
// sorted length is min(n, n_mul * *n_dev) (a count that lives on the device).
int64_t radix_hist_elems(int64_t n);
hipError_t radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n, int bits,
                            uint32_t* hist, uint32_t* scan_tmp, bool* result_in_1, hipStream_t s,
                            const uint32_t* n_dev = nullptr, uint32_t n_mul = 1);

hipError_t launch_lo_prep(const float* lo_V, int64_t nlv, const int32_t* lo_F, int64_t nlf,
                          const float* lo_UV, int32_t res, const Layout& L, char* ws,
                          hipStream_t s);
hipError_t launch_raster(int64_t nlf, int32_t res, const Layout& L, char* ws, hipStream_t s);
hipError_t launch_bvh_build(const float* hi_V, int64_t nhv, const int32_t* hi_F, int64_t nhf,
                            const Layout& L, char* ws, hipStream_t s);
hipError_t launch_traverse(const float* lo_V, const int32_t* lo_F, int64_t nlf,
                           const int32_t* hi_F, int64_t nhv, int64_t nhf, const float* hi_N,
                           float max_dist,
                           float* out_map, int32_t* out_hit, bool save, const TravConfig& cfg,
                           const Layout& L, char* ws, hipStream_t s);
hipError_t launch_fill_uncovered(int32_t res, float* out_map, int32_t* out_hit, const Layout& L,
                                 char* ws, hipStream_t s);
hipError_t launch_dilate(int32_t res, int passes, float* out_map, const Layout& L, char* ws,
                         hipStream_t s);
hipError_t launch_rgb8(int32_t res, const float* out_map, uint8_t* rgb, hipStream_t s);

hipError_t launch_backward(const float* hi_V, const int32_t* hi_F, int64_t nhv, const float* hi_N,
                           const float* lo_V, const int32_t* lo_F, int64_t nlv, int64_t nlf,
                           const float* grad_map, float* grad_lo_V, float* grad_hi_N, const Layout& L,
                           char* ws, hipStream_t s);
hipError_t launch_sq_loss(const float* map, const float* target, int64_t n3, float* grad, float* loss,
                          float* partial, hipStream_t s);

}  // namespace bake
