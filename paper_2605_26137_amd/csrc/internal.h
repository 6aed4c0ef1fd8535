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

// Full-precision box slots of a binary node, by child side (build scratch:
// the refit hands the boxes of the top levels over through these):
//   a = (L.lo.x, L.lo.y, L.lo.z, L.hi.x)
//   b = (L.hi.y, L.hi.z, R.lo.x, R.lo.y)
//   c = (R.lo.z, R.hi.x, R.hi.y, R.hi.z)
struct alignas(16) BvhNode {
    float4 a, b, c;
    int4 unused;
};
static_assert(sizeof(BvhNode) == 64, "BvhNode is 64 B");

// Binary BVH node as the traversal reads it (32 B, two 16-B loads per
// visit): the boxes of both children quantised to 8 bits per plane in a
// frame of the node's own.
//   a = (o.x, o.y, o.z, meta): meta byte k = biased exponent e_k of the axis-k
//       step 2^(e_k - 127)
//   q = (q0, q1, q2, child): the 12 bytes of q0..q2 in order are the planes
//       L.lo.xyz, L.hi.xyz, R.lo.xyz, R.hi.xyz; child = index g of the left
//       child (the right one is g + 1) with bit 30 / 31 set when the left /
//       right child is a leaf
// A plane with byte v decodes as fmaf(v, 2^(e_k - 127), o_k) in FP32; the
// build picks the bytes so that every decoded child box contains the child's
// box (a lower plane rounds down, an upper one up).  A node whose box is not
// finite on an axis decodes to NaN planes there, which the box tests treat as
// an unbounded slab.
struct alignas(16) BvhNodeC {
    float4 a;
    uint4 q;
};
static_assert(sizeof(BvhNodeC) == 32, "BvhNodeC is 32 B");
constexpr uint32_t kChildLeafL = 1u << 30, kChildLeafR = 1u << 31, kChildIndex = kChildLeafL - 1u;

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
                   kStInternal = 16u, kStState = 32u;

// Per-ray status values (mirror of bake.h).
constexpr int32_t kMiss = -1, kUnreliable = -2, kUncovered = -3;

// ---------------------------------------------------------------------------
// Batches.  Every launch works on a batch of assets (a single bake is a batch
// of one).  Per-element arrays of all assets are concatenated; each asset
// knows where its elements start.  A launch's blocks are split among the
// assets by a per-grid prefix table, so a block belongs to exactly one asset
// and finds it by a binary search over that table: a batched asset goes
// through exactly the arithmetic of a single bake.
// ---------------------------------------------------------------------------

struct AssetDev {
    const float* hi_V;
    const int32_t* hi_F;
    const float* hi_N;
    const float* lo_V;
    const int32_t* lo_F;
    const float* lo_UV;
    float* out_map;
    int32_t* out_hit;
    uint8_t* out_rgb8;  // may be null
    int32_t nhv, nhf, nlv, nlf;
    int32_t res, log2res;
    float max_dist;
    int32_t index;  // position in the batch
    // first element of this asset in the concatenated arrays
    int64_t lv;     // lo vertices
    int64_t lf;     // lo faces
    int64_t hf;     // hi triangles (sort keys, leaves)
    int64_t node;   // internal BVH nodes (nhf - 1 per asset)
    int64_t tex;    // texels
    int64_t stile;  // sort tiles of the BVH keys
    int64_t btile;  // sort tiles of the backward pairs (capacity 3 res^2)
    int64_t tl;     // treelet and frontier slots
};

// Inputs and outputs of the backward pass, one per asset.
struct AssetGrad {
    const float* grad_map;  // [res, res, 3]
    float* grad_lo_V;       // [nlv, 3] or null
    float* grad_hi_N;       // [nhv, 3] or null
};

// Grids: per-asset block counts of the launches, as prefix tables.
enum GridId : int {
    kGLoF = 0,  // lo faces, 256 per block
    kGLoFWave,  // lo faces, one wave each (4 per block)
    kGLoV,      // lo vertices, 256 per block
    kGHiV,      // hi vertices, 256 per block
    kGHiF,      // hi triangles, 256 per block
    kGSort,     // BVH sort tiles (kSortTile keys per block)
    kGTex,      // texels, 256 per block
    kGTex3,     // texel channels, 256 per block
    kGBwdSort,  // backward sort tiles (capacity 3 res^2, kSortTile per block)
    kGTile,     // kFinishTile^2 texel tiles of the fused uncovered fill + dilation
    kGridCount
};

constexpr int kSortTile = 4096;  // keys per radix-sort block and pass
constexpr int kBoundsSplit = 4;  // centroid-bounds workgroups per sort tile (a partial each)
constexpr int kSortPasses = 4;   // 8-bit digits of keys up to 32 bits
constexpr int kSuper = 32;       // sort tiles per super-tile (digit counts summed per super-tile)
// Super-tile rows of a sort over `tiles` tiles of `n` assets (asset a's rows
// start at its first tile / kSuper + a).
__host__ __device__ inline int64_t sort_super_rows(int64_t tiles, int64_t n) { return tiles / kSuper + n + 1; }
constexpr int kFinishTile = 56;  // texel tile side of the fused fill + dilation (tile + 2 halos <= 64)
constexpr int kMaxFusedPasses = 4;  // more dilation passes run one launch per pass

// Treelet and frontier capacity per asset.  Treelet roots are the small
// children of the nodes with more than 2048 leaves ("big" nodes).  Big nodes
// whose children are both small cover disjoint ranges of > 2048 leaves, so
// there are fewer than n / 2048 of them, and every big node lies on the root
// path (at most 62 nodes) of one of them: fewer than 62 n / 2048 + 62 big
// nodes, one more treelet than big nodes.
__host__ __device__ inline int64_t treelet_cap(int64_t n) { return n / 32 + 2 * kMaxDepth + 16; }

// Per-asset counter slots.
constexpr int kCntRays = 0;      // covered texels (rays)
constexpr int kCntBoxLo = 2;     // u64 box tests (FLAG_COUNT), slots 2-3
constexpr int kCntTriLo = 4;     // u64 triangle tests (FLAG_COUNT), slots 4-5
constexpr int kCntFrontier = 6;  // refit frontier length
constexpr int kCntTreelets = 7;  // refit treelets
constexpr int kCntIterLo = 8;    // u64 traversal loop trips of whole waves (FLAG_COUNT), slots 8-9
constexpr int kCntTop = 10;      // refit top nodes (internal nodes above the treelets)
constexpr int kCntSlots = 16;
// Batch counter slots.
constexpr int kGcQueue = 0;  // traversal work queue head
constexpr int kGcSeal = 1;   // nonce of the last forward with BAKE_FLAG_SAVE (written as it starts; 0 after one without)
constexpr int kGcBwdTiles = 2;  // backward sort tiles that hold pairs, over the batch (written after the raster)
constexpr int kXcds = 8;         // XCDs of an MI355X: each has its own L2
constexpr int kXcdStride = 32;   // one 128-byte line per XCD queue head
constexpr int kGcXcdQueue = 32;  // kXcds traversal queue heads, kXcdStride apart
constexpr int kGcSlots = kGcXcdQueue + kXcds * kXcdStride;

// What every kernel receives: the asset table and the batch-wide tables.
struct Batch {
    const AssetDev* A;      // [n]
    const AssetGrad* G;     // [n] (backward only)
    const int32_t* gpf;     // [kGridCount][n + 1] block prefix of each grid
    const uint32_t* ray_pf; // [n + 1] first ray of each asset (written after the raster)
    const uint32_t* rb_pf;  // [n + 1] 64-ray batches before each asset
    const uint32_t* tl_pf;  // [n + 1] treelets before each asset
    const uint32_t* bt_pf;  // [n + 1] backward sort tiles holding pairs before each asset (after the raster)
    uint32_t* cnt;          // [n][kCntSlots]
    uint32_t* gcnt;         // [kGcSlots]
    uint32_t* status;       // status word, OR over the batch
    int n;
    uint32_t seal;          // backward: the nonce the saved forward left in gcnt[kGcSeal]
};

// Backward kernels run only on the state of the forward they were planned
// for: anything else (a workspace reused since) makes them do nothing.
__device__ __forceinline__ bool sealed(const Batch& B) {
    if (B.gcnt[kGcSeal] == B.seal) return true;
    if (threadIdx.x == 0 && blockIdx.x == 0) atomicOr(B.status, kStState);
    return false;
}

// Last index a in [0, n) with p[a] <= x (p ascending, p[0] <= x).
template <typename T>
__device__ __forceinline__ int upper_asset(const T* p, int n, int64_t x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)p[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Asset and asset-local block index of block `blk` of grid g.
__device__ __forceinline__ int block_asset(const Batch& B, int g, int64_t blk, int64_t* local) {
    const int32_t* p = B.gpf + (int64_t)g * (B.n + 1);
    const int a = upper_asset(p, B.n, blk);
    *local = blk - p[a];
    return a;
}

__device__ __forceinline__ void set_status(const Batch& B, uint32_t bits) { atomicOr(B.status, bits); }

// Host description of a batch: asset table, grid prefix tables and the
// workspace layout.
struct Layout {
    size_t status, counters, gcnt, table, grads, gpf, ray_pf, rb_pf, tl_pf, bt_pf;
    size_t lo_n, lo_deg, lo_off, lo_cur, lo_adj;  // lo vertex normals + vertex->face CSR
    size_t face_t, face_uv, face_cnt, face_off;   // per lo face
    size_t scan_tmp;                              // block sums of the scans
    size_t facemap, level;                        // per texel
    size_t rays, hits;                            // per ray
    size_t bounds_part, bounds;                   // centroid bounds: per sort tile, per asset
    size_t keys0, keys1, vals0, vals1, hist, sup; // radix sort of the BVH keys
    size_t nodes, nodes_c, leaves, node_parent, leaf_parent, refit_cnt, frontier, treelets, top, child;
    size_t spill;                                 // traversal stack spill
    // backward scratch (BAKE_FLAG_SAVE only)
    size_t bwd_ray, bwd_hterm, bwd_k0, bwd_v0, bwd_k1, bwd_v1, bwd_hist, bwd_sup, bwd_face1, bwd_face2, bwd_sbar,
        bwd_vbar;
    size_t total;
    // batch totals
    int n;
    int64_t t_lv, t_lf, t_hv, t_hf, t_node, t_tex, t_stile, t_btile, t_tl;
    int64_t spill_lanes, scan_tmp_n;
    int max_hv_bits;  // bit length of the largest nhv (backward sort keys lie in [0, nhv])
    bool save;
};

struct BatchHost {
    Layout L;
    const AssetDev* A = nullptr;  // [n] host copy of the table
    const int32_t* gpf = nullptr; // [kGridCount][n + 1] host copy
    char* ws = nullptr;           // device workspace
    Batch dev;                    // kernel view (device pointers)
    int64_t blocks(int g) const { return gpf[(int64_t)g * (L.n + 1) + L.n]; }
};

// Traversal configuration
struct TravConfig {
    int block;    // 64 / 128 / 256
    int stack;    // LDS entries per lane: 8 / 16 / 32
    int mode;     // 0: 64-ray batches, mixed trips; 1: lane refill from a ray queue;
                  // 2: 64-ray batches, internal-node and leaf phases;
                  // 3: 64-ray batches, balanced all-node / all-leaf trips
    bool count = false;    // instrumented variant: count box and triangle tests
    bool closest = false;  // closest-point query instead of the ray query
    bool xcd = true;       // wave batches: one work queue per XCD (traverse.hip)
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

// Copies `bytes` host bytes to device memory through by-value kernel
// arguments (no host-to-device copy, so it can be recorded in a graph).
// With zero_words > 0, the first launch also zeroes zero[0, zero_words),
// except word set_idx, which takes set_val.
hipError_t write_table(void* dst, const void* src, size_t bytes, hipStream_t s, uint32_t* zero = nullptr,
                       int64_t zero_words = 0, int64_t set_idx = -1, uint32_t set_val = 0);
// The backward sort's super-tile rows, which its caller zeroes before the sort.
int64_t bwd_sort_zero_words(const Layout& L);

// Per-asset ray starts, 64-ray batch prefix and backward sort tile prefix
// (after the raster); treelet prefix (after the hierarchy kernel has listed
// the treelets).
hipError_t launch_ray_spaces(const BatchHost& H, hipStream_t s);
hipError_t launch_treelet_space(const BatchHost& H, hipStream_t s);

// Stable LSD radix sort of every asset's (key, value) pairs on the low `bits`
// bits, 8 per pass, ping-ponging between the two buffers of the sort:
// kSortBvh: the Morton keys (keys0/vals0 <-> keys1/vals1); kSortBwd: the
// backward pairs (bwd_k0/bwd_v0 <-> bwd_k1/bwd_v1), three per ray.
// *result_in_1 tells which buffer holds the result (the same for all assets).
enum SortWhich : int { kSortBvh = 0, kSortBwd = 1 };
// after_first: if not null, recorded on s once the first pass's histogram is
// queued (or at once when there is nothing to sort).
hipError_t launch_sort(const BatchHost& H, int which, int bits, bool* result_in_1, hipStream_t s,
                       hipEvent_t after_first = nullptr);

hipError_t launch_lo_prep(const BatchHost& H, hipStream_t s);
hipError_t launch_raster(const BatchHost& H, hipStream_t s);
hipError_t launch_fill_uncovered(const BatchHost& H, hipStream_t s);
hipError_t launch_bvh_build(const BatchHost& H, hipStream_t s);
hipError_t launch_traverse(const BatchHost& H, const TravConfig& cfg, hipStream_t s);

// Hidden-face removal (Sec. 6.2) on the BVH of asset 0 of a planned batch.
struct VisRun {
    const float* eyes;   // device [n_views][3]
    float target[3];
    float tan_half;
    int32_t n_views, res;
    uint32_t* visible;   // device [n_f] flags, set to 1 for every first-hit face
    int32_t* first_hit;  // NULL or device [n_views res^2]
    float* depth;        // NULL or device [n_views res^2]: first-hit distance along the ray, +inf none
    int32_t* spill;      // [kMaxDepth][spill_lanes]
    int64_t spill_lanes;
    bool count;          // instrumented: box / triangle tests and wave trips into asset 0's counters
};
hipError_t launch_visibility_rays(const BatchHost& H, const VisRun& v, hipStream_t s);
// Backprojection precompute (Sec. 7.4, TextureGen Postprocessing) for asset
// 0's covered texels (its ray list and low-poly normals) against the depth
// buffers of the views.
struct MapRun {
    const float* eyes;  // device [n_views][3]
    float target[3];
    float tan_half;
    int32_t n_views, img_res;
    const float* depth;  // device [n_views][img_res^2]: first-hit distances along the pixel rays
    float tol;
    float* uv_out;       // device [n_views][res^2][2], pre-filled with -1
    float* inc_out;      // device [n_views][res^2], pre-filled with 0
};
hipError_t launch_view_maps(const BatchHost& H, const MapRun& m, hipStream_t s);
// Vertex -> face lists and the normal-gated flood fill from `visible` into
// `ext` (both [n_f] u32 flags), then both written out as bytes.
struct FillRun {
    uint32_t *deg, *off, *cur, *adj, *ext, *front0, *front1, *scan_tmp;
    const uint32_t* visible;
    uint8_t *visible_out, *exterior_out;
};
hipError_t launch_flood_fill(const BatchHost& H, const FillRun& f, hipStream_t s);
// Quadric edge-collapse simplification (Sec. 6.1): workspace carving and the
// two blocking drivers (they synchronise `s` to read the per-round counts).
struct QemLayout {
    int64_t nv, nf, edge_cap;
    size_t cnt, hist, P, Q, P2, Q2, F, F2, keep, koff, deg, off, cur, adj, ncnt, noff, hcnt, eoff, bnd, nbr, keep_ring, E, bits, faces,
        pl, m, M, partner, wflag, part, scan_tmp;
    size_t total;
};
size_t qem_layout(int64_t nv, int64_t nf, QemLayout* L);
// Edges of the input mesh with their collapse evaluated; *status != 0 flags
// bad faces, *n_edges > cap leaves the outputs untouched.
hipError_t qem_edges_run(const QemLayout& L, char* ws, const float* V, const int32_t* F, int midpoint,
                         double* Q_out, int64_t cap, int32_t* E_out, uint8_t* valid_out, int32_t* faces_out,
                         double* cost_out, double* p_out, uint32_t* status, int64_t* n_edges, hipStream_t s);
hipError_t qem_simplify_run(const QemLayout& L, char* ws, const float* V, const int32_t* F, int64_t target, double rho,
                            int32_t max_rounds, int midpoint, float* V_out, int32_t* F_out, int64_t* counts,
                            int32_t* rounds_out, int64_t* stats, float* times_ms, uint32_t* status, hipStream_t s);
hipError_t launch_dilate(const BatchHost& H, int passes, hipStream_t s);
hipError_t launch_rgb8(const BatchHost& H, hipStream_t s);
// With `side` (and its fork / join events), the low-poly gradient chain runs on
// `side` beside the high-poly one and joins `s` before the call returns.
hipError_t launch_backward(const BatchHost& H, bool any_lo, bool any_hi, hipStream_t s, hipStream_t side = nullptr,
                           hipEvent_t fork = nullptr, hipEvent_t join = nullptr);
hipError_t launch_sq_loss(const float* map, const float* target, int64_t n3, float* grad, float* loss,
                          float* partial, hipStream_t s);

}  // namespace bake
