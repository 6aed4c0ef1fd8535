/*
 * bake.h -- C ABI of the MI355X (gfx950) tangent-space normal baker.
 *
 * The operation is the paper's normal-map bake (Sec. 6.4 "Normal Map Baking"):
 * the low-poly mesh is rasterised into its own UV atlas, giving per covered
 * texel a world position, an interpolated smooth normal and a tangent frame;
 * a BVH over the high-poly mesh finds the corresponding high-poly point; the
 * high-poly smooth normal is interpolated there with barycentric weights,
 * projected into the texel's tangent frame and written to the map; far or
 * unreliable correspondences get the neutral normal (0,0,1); finally charts
 * are dilated so mip filtering does not bleed background into them.
 *
 * The correspondence query here is a two-sided ray cast from the texel's world
 * position along its interpolated low-poly normal: the hit with the smallest
 * |t| for t in [-max_dist, +max_dist], ties to the lower high-poly triangle
 * index.  (The paper's variant queries the closest surface point and filters
 * at 1% of the bounding-box diagonal; `max_dist` takes that filter's role.)
 *
 * Conventions shared by every entry point:
 *   - All array pointers are DEVICE pointers (hipMalloc / torch CUDA tensors),
 *     contiguous, row-major, owned by the caller.  The library never frees them
 *     and keeps no reference after the call returns.
 *   - No hidden device allocation: scratch memory is the caller's `workspace`
 *     (size from bake_workspace_size).  Everything is enqueued asynchronously
 *     on `stream` (a hipStream_t; NULL = the default stream) and returns
 *     without synchronising, except bake_query_status / bake_read_counter.
 *   - Texel (i, j) is row i, column j of a [res][res] image; its centre is
 *     u = (j + 1/2)/res, v = (i + 1/2)/res.
 *   - Per-corner UVs are snapped to 1/256 texel; a texel is covered by a face
 *     when its centre is inside or on the snapped UV triangle (either
 *     orientation); on overlap the lowest face index wins.
 *   - Return value: BAKE_OK (0) or a negative BAKE_E_* code; a message is kept
 *     in a thread-local buffer (bake_last_error).  Argument errors are detected
 *     on the host before any work is enqueued.
 */
#ifndef PAPER_2605_26137_AMD_BAKE_H
#define PAPER_2605_26137_AMD_BAKE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------- */
#define BAKE_OK 0
#define BAKE_E_INVALID_ARG -1 /* null pointer, negative count, bad max_dist, ... */
#define BAKE_E_UNSUPPORTED -2 /* res not a power of two in [1, 16384], size limits */
#define BAKE_E_WORKSPACE -3   /* workspace missing, too small or misaligned */
#define BAKE_E_INDEX -4       /* device status word reported bad input data */
#define BAKE_E_HIP -5         /* a HIP runtime call failed */
#define BAKE_E_STATE -6       /* backward called without a saved forward */

/* ---- per-texel status written to out_hit ----------------------------- */
/* >= 0: index of the high-poly triangle that was hit (original hi_F order) */
#define BAKE_MISS -1       /* no high-poly surface within +-max_dist */
#define BAKE_UNRELIABLE -2 /* degenerate UV/3D face, zero normal or tangent parallel to the normal */
#define BAKE_UNCOVERED -3  /* no low-poly face covers the texel centre */

/* ---- device status word bits (bake_query_status) --------------------- */
#define BAKE_STATUS_LO_INDEX 1u  /* lo_F index outside [0, n_lo_v) */
#define BAKE_STATUS_HI_INDEX 2u  /* hi_F index outside [0, n_hi_v) */
#define BAKE_STATUS_BAD_UV 4u    /* UV non-finite or outside [-1, 2]; face skipped */
#define BAKE_STATUS_NONFINITE 8u /* non-finite vertex position; face/triangle skipped */
#define BAKE_STATUS_INTERNAL 16u /* internal consistency guard tripped (should never happen) */
#define BAKE_STATUS_STATE 32u    /* a backward found the workspace no longer holding the saved
                                    forward's state (reused since): it wrote nothing */

/* ---- correspondence query (bake_options.query) ------------------------ */
#define BAKE_QUERY_RAY 0     /* two-sided ray along the interpolated low-poly normal: the
                                hit with the smallest |t| in [-max_dist, +max_dist]       */
#define BAKE_QUERY_CLOSEST 1 /* the paper's own form (Sec. 6.4): the closest point of the
                                high-poly surface within max_dist (the paper's bound is 1%
                                of the bounding-box diagonal); ties within one distance
                                quantum max_dist*2^-20 go to the lower triangle index.
                                Forward only: BAKE_FLAG_SAVE is rejected (BAKE_E_UNSUPPORTED);
                                trav_mode 1 runs as 3.                                     */

/* ---- flags ------------------------------------------------------------ */
#define BAKE_FLAG_SAVE 1u   /* keep the per-ray state that bake_normals_backward needs */
#define BAKE_FLAG_TIMING 2u /* record per-stage HIP events (bake_stage_times) */
#define BAKE_FLAG_COUNT 4u  /* instrumented traversal: count box and triangle tests
                               (bake_read_counter 1 and 2); slower, same results */
#define BAKE_FLAG_ONE_STREAM 8u /* run every stage on the caller's stream: no second
                                   stream for the low-poly work beside the BVH build
                                   (forward) and the high-poly sort (backward); the
                                   backward of a saved forward follows the forward's
                                   choice.  Same results bit for bit.              */
#define BAKE_FLAG_ONE_QUEUE 16u /* the ray traversal's persistent waves take their
                                   (asset, 64-ray batch) items from one work queue
                                   in face order, instead of the default of one
                                   queue per XCD over a contiguous part of the items
                                   (the waves sharing an L2 then trace one region of
                                   the surface).  Same results bit for bit.         */

typedef struct bake_options {
    int32_t dilate_passes; /* chart dilation passes, 0..64 (default 2)                    */
    uint32_t flags;        /* BAKE_FLAG_*                                                  */
    uint8_t *out_rgb8;     /* optional device [res,res,3] u8 map: floor((x+1)*127.5+0.5)   */
    int32_t trav_block;    /* traversal workgroup size: 64, 128, 256 (0 = tuned default)  */
    int32_t trav_stack;    /* LDS stack entries per lane: 8, 16, 32 (0 = tuned default)    */
    int32_t trav_mode;     /* persistent waves; 0 = whole 64-ray batches, each loop trip
                              a step of either kind per lane; 1 = finished lanes
                              refilled from a ray queue; 2 = whole 64-ray batches,
                              internal nodes and leaves in separate phases; 3 = whole
                              64-ray batches, each trip all-internal or all-leaf, a
                              leaf trip once half the busy lanes wait at a leaf;
                              -1 = default (3).  Results do not depend on it.           */
    int32_t query;         /* BAKE_QUERY_RAY (default) or BAKE_QUERY_CLOSEST                 */
    int32_t reserved[3];
} bake_options;

/* Default options: dilate_passes = 2, no flags, no RGB8, tuned traversal. */
void bake_default_options(bake_options *opt);

/* Workspace bytes needed for a bake of these sizes with these options (NULL =
 * defaults).  The workspace must be device memory aligned to 256 bytes. */
int32_t bake_workspace_size(int64_t n_hi_v, int64_t n_hi_f, int64_t n_lo_v, int64_t n_lo_f,
                            int32_t res, const bake_options *opt, size_t *bytes_out);

/* Forward bake (Sec. 6.4, four stages: UV rasterisation to a G-buffer, BVH
 * build over the high-poly, per-texel correspondence query with distance and
 * UV-reliability filters, tangent-space projection and seam dilation).
 *
 *   hi_V  [n_hi_v,3] f32  high-poly vertex positions
 *   hi_F  [n_hi_f,3] i32  high-poly triangles (indices into hi_V)
 *   hi_N  [n_hi_v,3] f32  high-poly smooth vertex normals (need not be unit)
 *   lo_V  [n_lo_v,3] f32  low-poly vertex positions
 *   lo_F  [n_lo_f,3] i32  low-poly triangles
 *   lo_UV [n_lo_f,3,2] f32 per-corner UVs, nominally in [0,1]
 *   res   atlas side, a power of two in [1, 16384]
 *   max_dist  finite, > 0: query range along the ray, both directions
 *   out_map [res,res,3] f32  tangent-space normal (T', B', N) components
 *   out_hit [res,res]   i32  hit triangle id or BAKE_MISS/UNRELIABLE/UNCOVERED
 *
 * Low-poly vertex normals are not an input: they are the normalised
 * area-weighted sums of incident face normals.  The per-face tangent comes from
 * the snapped UV derivatives; per texel it is made orthogonal to the
 * interpolated normal N, and the bitangent is h_f (N x T') with h_f the face's
 * UV handedness.  Uncovered texels are (0,0,1) before dilation; dilation fills
 * them from covered neighbours and leaves their id at BAKE_UNCOVERED.
 * Bad index data does not fault: offending faces are skipped and a bit is set
 * in the device status word (bake_query_status). */
int32_t bake_normals(const float *hi_V, int64_t n_hi_v, const int32_t *hi_F, int64_t n_hi_f,
                     const float *hi_N, const float *lo_V, int64_t n_lo_v, const int32_t *lo_F,
                     int64_t n_lo_f, const float *lo_UV, int32_t res, float max_dist,
                     float *out_map, int32_t *out_hit, const bake_options *opt, void *workspace,
                     size_t workspace_bytes, void *stream);

/* Backward of L(out_map before dilation) with the hit selection, the texel ->
 * face assignment and the handedness held fixed: given grad_map = dL/dout_map
 * [res,res,3], writes dL/dlo_V [n_lo_v,3] and dL/dhi_N [n_hi_v,3] (both
 * overwritten, not accumulated).  Only texels with a hit carry gradient;
 * misses, unreliable, uncovered and dilated texels are constants.  (The paper
 * has no backward pass; this differentiates its bake as defined above.)
 * Needs the workspace of the last forward call made with BAKE_FLAG_SAVE on the
 * same inputs (else BAKE_E_STATE); the workspace size is the one of that
 * forward.  That forward leaves a nonce in the workspace; if the memory was
 * overwritten since, the backward kernels find a different value, write
 * nothing and set BAKE_STATUS_STATE.  Sums are done in a fixed order
 * (no floating-point atomics): the result is bitwise reproducible.  Either
 * gradient pointer may be NULL to skip it. */
int32_t bake_normals_backward(const float *hi_V, int64_t n_hi_v, const int32_t *hi_F,
                              int64_t n_hi_f, const float *hi_N, const float *lo_V, int64_t n_lo_v,
                              const int32_t *lo_F, int64_t n_lo_f, const float *lo_UV, int32_t res,
                              float max_dist, const float *grad_map, float *grad_lo_V,
                              float *grad_hi_N, void *workspace, size_t workspace_bytes,
                              void *stream);

/* ---- the forward bake without a workspace -------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * forward bake as bake_normals, same arguments minus the workspace, with the
 * scratch memory taken from a fixed array of BAKE_NOALLOC_BYTES inside the
 * library's device code, one per GPU, held until the process ends.  The call
 * allocates no device memory (no hipMalloc / hipFree and no library routine
 * that allocates device memory; host-side planning uses small host
 * containers).  Its results are bitwise those of bake_normals on the same
 * inputs and options.
 *   - Limit: a bake whose bake_workspace_size exceeds BAKE_NOALLOC_BYTES fails
 *     with BAKE_E_WORKSPACE before anything is enqueued (128 MiB holds, e.g.,
 *     a 512^2 atlas over a 327,680-triangle high-poly; use bake_normals for
 *     larger bakes).
 *   - opt->flags may not hold BAKE_FLAG_SAVE, BAKE_FLAG_TIMING or
 *     BAKE_FLAG_COUNT (BAKE_E_INVALID_ARG): the saved state, the counters and
 *     the status word stay in the shared array, which no other entry point
 *     can name.  Every stage runs on `stream` (BAKE_FLAG_ONE_STREAM implied).
 *   - All calls on one GPU share that GPU's array and it keeps the last
 *     call's contents; each call clears what must start at zero.  Calls that
 *     overlap on one GPU (other streams, other threads) RACE: serialise them.
 *   - The first call on a device resolves the array's device address (a
 *     runtime query, made once per device with that device current).
 * Bad index data does not fault (as for bake_normals), but the device status
 * word is not readable from here. */
#define BAKE_NOALLOC_BYTES (128u << 20)
int32_t bake_normals_noalloc(const float *hi_V, int64_t n_hi_v, const int32_t *hi_F, int64_t n_hi_f,
                             const float *hi_N, const float *lo_V, int64_t n_lo_v, const int32_t *lo_F,
                             int64_t n_lo_f, const float *lo_UV, int32_t res, float max_dist,
                             float *out_map, int32_t *out_hit, const bake_options *opt, void *stream);

/* ---- hidden-face removal (Sec. 6.2) ------------------------------------ */
/* Visibility rays from viewpoints around a mesh, then a flood fill that
 * propagates "exterior" across shared edges (the paper's pass that finds the
 * interior faces of a generated mesh: 512 viewpoints on a surrounding sphere,
 * 1024-pixel images, a face is visible when some ray reaches it unoccluded;
 * the fill starts from the visible faces and crosses an edge only when the
 * two faces' normals agree in direction).
 *
 * Cameras: view v is a pinhole at eyes[v] looking at target (3 floats, HOST
 * pointer); with forward f = normalise(target - eye), helper a = the world
 * axis with the smallest |target_k - eye_k| (lowest k on ties, decided on the
 * exact differences), right r = normalise(f x a),
 * up u = r x f, pixel (i, j) of the res x res image looks along
 * normalise(f + x r + y u), x = ((j + 1/2) 2/res - 1) tan_half_fov,
 * y = (1 - (i + 1/2) 2/res) tan_half_fov.  A ray's first hit is the face
 * minimising (floor(t / w), index), w = t_far 2^-20, over the faces it
 * crosses at 0 < t <= t_far with every barycentric weight >= -2^-14 (the
 * bake's hit rule on the half-line).
 * Flood fill: faces f, g sharing two distinct vertex indices; g joins from
 * an exterior f when n_f . n_g > 0, n = (V1 - V0) x (V2 - V0) in FP64 from
 * the float vertices (no fused operations).
 *
 * V [n_v,3] f32, F [n_f,3] i32, eyes [n_views,3] f32: device.  Outputs
 * (device, caller-owned): visible_out [n_f] u8 (1 = some ray's first hit),
 * exterior_out [n_f] u8 or NULL (visible faces and every face the fill
 * reaches), first_hit_out NULL or [n_views][res][res] i32 (first hit id, -1
 * none).  flags: BAKE_FLAG_COUNT (box / triangle tests and wave trips of the
 * camera rays, bake_read_counter 1-3), BAKE_FLAG_TIMING (bake_stage_times:
 * setup, BVH build, rays, flood fill, -, total).  The workspace (>=
 * bake_visibility_workspace_size bytes, 256-byte aligned) is overwritten; no
 * device memory is allocated.  Indices outside [0, n_v) raise
 * BAKE_STATUS_HI_INDEX (the face is never hit and never joins the fill).
 * Errors: BAKE_E_INVALID_ARG (NULL pointers, n_views outside [1, 2^20], res
 * outside [1, 16384], non-finite or non-positive tan_half_fov / t_far),
 * BAKE_E_UNSUPPORTED (counts >= 2^30), BAKE_E_WORKSPACE. */
int32_t bake_visibility_workspace_size(int64_t n_v, int64_t n_f, size_t *bytes_out);
int32_t bake_visibility(const float *V, const int32_t *F, int64_t n_v, int64_t n_f, const float *eyes,
                        int32_t n_views, const float *target, float tan_half_fov, int32_t res, float t_far,
                        uint32_t flags, uint8_t *visible_out, uint8_t *exterior_out, int32_t *first_hit_out,
                        void *workspace, size_t workspace_bytes, void *stream);

/* ---- backprojection precompute (Sec. 7.4, TextureGen Postprocessing) ---- */
/* The per-texel, per-view data that backprojecting K generated views onto a
 * UV atlas needs: the paper recovers each atlas texel's surface point,
 * projects it into every view, weights a view by the incidence between the
 * surface normal and the viewing direction, and zeroes that weight where a
 * depth-buffer test finds the point occluded beyond a fixed tolerance.
 *
 * The atlas is rasterised exactly as the bake's low-poly (texel centres,
 * 1/256-texel snapped UVs, lowest face on overlaps); a covered texel's surface
 * point p and unit smooth normal n (interpolated area-weighted vertex
 * normals) are the bake's G-buffer.  Views are the pinholes of
 * bake_visibility (eyes, target, tan_half_fov, img_res x img_res pixels).
 * Depth buffer of view k: per pixel, the view-axis depth t (d . f) of the
 * pixel ray's first hit on the mesh (+inf where it hits nothing, t in
 * (0, t_far]); depth_out receives the hit distances t themselves.  Per texel and view, with q = p - e_k and z = q . f:
 *   image coordinates col = (q.r / (z tan_half) + 1) img_res / 2 - 1/2,
 *   row = (1 - q.u / (z tan_half)) img_res / 2 - 1/2 (pixel centres at
 *   integers), or (-1, -1) when z <= 0 or either lies outside
 *   [-1/2, img_res - 1/2);
 *   incidence max(0, n . (e_k - p) / |e_k - p|), or 0 when outside, when the
 *   normal is undefined, or when z > depth[nearest pixel] + depth_tol.
 *
 * V [n_v,3] f32, F [n_f,3] i32, UV [n_f,3,2] f32 (per corner), eyes
 * [n_views,3] f32: device.  target: HOST pointer to 3 floats.  Outputs
 * (device, caller-owned): uv_out [n_views][res*res][2] f32 (col, row),
 * inc_out [n_views][res*res] f32 (uncovered texels: (-1, -1) and 0),
 * depth_out NULL or [n_views][img_res][img_res] f32 (first-hit distance t of
 * each pixel ray, +inf for none).  flags: BAKE_FLAG_COUNT
 * (box / triangle tests and wave trips of the depth rays, bake_read_counter
 * 1-3), BAKE_FLAG_TIMING (bake_stage_times: G-buffer, BVH build, depth rays,
 * maps, -, total).
 * Workspace >= bake_view_maps_workspace_size bytes, 256-byte aligned,
 * overwritten; nothing is allocated.  Errors: BAKE_E_INVALID_ARG (NULL
 * pointers, n_views outside [1, 4096], img_res outside [1, 16384], non-finite
 * or non-positive tan_half_fov / t_far, negative depth_tol), BAKE_E_UNSUPPORTED
 * (res not a power of two in [1, 16384], counts >= 2^30), BAKE_E_WORKSPACE. */
int32_t bake_view_maps_workspace_size(int64_t n_v, int64_t n_f, int32_t res, int32_t n_views, int32_t img_res,
                                      size_t *bytes_out);
int32_t bake_view_maps(const float *V, const int32_t *F, const float *UV, int64_t n_v, int64_t n_f, int32_t res,
                       const float *eyes, int32_t n_views, const float *target, float tan_half_fov,
                       int32_t img_res, float t_far, float depth_tol, uint32_t flags, float *uv_out,
                       float *inc_out, float *depth_out, void *workspace, size_t workspace_bytes, void *stream);

/* Squared-error map loss, a helper for training-style use of the backward:
 * loss_out[0] = sum_i (map[i] - target[i])^2 and, if grad_out is not NULL,
 * grad_out[i] = 2 (map[i] - target[i]), over n floats (n = res*res*3 for a map).
 * Device pointers; the sum is reduced in a fixed order (deterministic).
 * scratch: device memory of at least 4 * (ceil(n / 256) + 1) bytes. */
int32_t bake_sq_loss(const float *map, const float *target, int64_t n, float *grad_out,
                     float *loss_out, void *scratch, size_t scratch_bytes, void *stream);

/* Synchronises `stream` and returns the OR of BAKE_STATUS_* bits raised by the
 * last bake that used `workspace`. */
int32_t bake_query_status(const void *workspace, void *stream, uint32_t *status_out);

/* Synchronises `stream` and returns a device counter of the last bake that used
 * `workspace`: which = 0 -> number of covered texels (rays traced); 1 -> box
 * tests and 2 -> triangle tests of the traversal; 3 -> traversal loop trips
 * of whole 64-lane waves (1-3: bakes with BAKE_FLAG_COUNT).  A ray takes one
 * trip per internal node (two box tests) or leaf (one triangle test), so
 * (box / 2 + tri) / (64 * trips) is the fraction of lanes doing useful work. */
int32_t bake_read_counter(const void *workspace, int32_t which, void *stream, int64_t *value_out);

/* Location of an internal array inside the workspace, for inspection by tests
 * and tools: which = BAKE_VIEW_*.  Returns byte offset and byte size. */
#define BAKE_VIEW_RAYS 0     /* [n_rays] {i32 texel, i32 lo face, f32 b1, f32 b2}, face order */
#define BAKE_VIEW_HITS 1     /* [n_rays] {f32 t, f32 beta1, f32 beta2, i32 id} (FLAG_SAVE)   */
#define BAKE_VIEW_FACEMAP 2  /* [res*res] i32 covering face or INT32_MAX                      */
#define BAKE_VIEW_LO_N 3     /* [n_lo_v] {f32 x, y, z, valid}                                 */
#define BAKE_VIEW_SORTED 4   /* [n_hi_f] u32 Morton keys, sorted                              */
#define BAKE_VIEW_NODES 5    /* [n_hi_f-1] 32 B BVH nodes: frame origin (3 f32), per-axis
                                step exponents (u8 x 3), 8-bit child planes (L.lo, L.hi,
                                R.lo, R.hi, xyz each), left child index | leaf flags (bit
                                30 left, 31 right); plane = fmaf(byte, 2^(e-127), origin) */
#define BAKE_VIEW_LEAVES 6   /* [n_hi_f] 48 B leaf triangles: 3 vertices + original index      */
#define BAKE_VIEW_FACE_T 7   /* [n_lo_f] {f32 Tx, Ty, Tz, h}                                   */
#define BAKE_VIEW_SORTED_IDX 8 /* [n_hi_f] u32 triangle indices in the sorted key order      */
int32_t bake_workspace_view(int64_t n_hi_v, int64_t n_hi_f, int64_t n_lo_v, int64_t n_lo_f,
                            int32_t res, const bake_options *opt, int32_t which,
                            size_t *offset_out, size_t *bytes_out);

/* Per-stage GPU times in ms of the last bake on this thread made with
 * BAKE_FLAG_TIMING, from HIP events recorded on the bake's stream
 * (synchronises on those events).  Stages: 0 lo prep, 1 raster (+ uncovered
 * fill), 2 BVH build, 3 traversal + encode, 4 dilation (+ RGB8), 5 whole
 * forward.  For batches of at least 65,536 high-poly faces the lo prep and
 * raster run beside the BVH build on a second stream of the library (forked
 * from and joined to the bake's stream by events; created on the device's
 * first such forward that is not being graph captured): stage 2 then spans
 * from the start of the bake to the end of all three.  Returns the number of
 * stages written. */
int32_t bake_stage_times(float *ms_out, int32_t n);

/* The same for up to the 64 most recent timed bakes on this thread, oldest
 * first: ms_out is [max_bakes][6].  Returns the number of bakes written. */
int32_t bake_stage_history(float *ms_out, int32_t max_bakes);

/* ---- batches: many bakes in one launch sequence ------------------------
 *
 * A batch runs the same stages as bake_normals for every asset, each stage as
 * one set of launches over all assets: per-asset BVHs built together (sort
 * tiles never straddle two assets), one traversal over a device work queue of
 * (asset, 64-ray batch) items, and the backward likewise.  Every asset goes
 * through exactly the arithmetic of a single bake, so a batched asset's
 * outputs are bitwise equal to those of bake_normals / bake_normals_backward
 * on the same inputs.  The calls enqueue kernels only (the asset table is
 * passed as kernel arguments, no host-to-device copy), so a sequence of them
 * can be recorded into a HIP graph and replayed while the pointers stay
 * valid.  The batch's size limits: n_assets in [1, 65536]; every per-asset
 * limit of bake_normals; 3 * sum(res^2) < 2^32 and sum(n_hi_f) < 2^31. */
typedef struct bake_asset {
    const float *hi_V;     /* [n_hi_v,3] */
    int64_t n_hi_v;
    const int32_t *hi_F;   /* [n_hi_f,3] */
    int64_t n_hi_f;
    const float *hi_N;     /* [n_hi_v,3] */
    const float *lo_V;     /* [n_lo_v,3] */
    int64_t n_lo_v;
    const int32_t *lo_F;   /* [n_lo_f,3] */
    int64_t n_lo_f;
    const float *lo_UV;    /* [n_lo_f,3,2] */
    int32_t res;
    float max_dist;
    float *out_map;        /* [res,res,3] */
    int32_t *out_hit;      /* [res,res] */
    uint8_t *out_rgb8;     /* optional [res,res,3] */
    const float *grad_map; /* backward input  [res,res,3] */
    float *grad_lo_V;      /* backward output [n_lo_v,3] or NULL */
    float *grad_hi_N;      /* backward output [n_hi_v,3] or NULL */
} bake_asset;

/* Workspace bytes for a batch (opt as for bake_normals; opt->out_rgb8 must be
 * NULL: RGB8 outputs are per asset). */
int32_t bake_batch_workspace_size(const bake_asset *assets, int32_t n_assets, const bake_options *opt,
                                  size_t *bytes_out);

/* Forward bake of every asset of the batch (bake_normals semantics per asset;
 * outputs through each asset's out_map / out_hit / out_rgb8).  The device
 * status word is the OR over the batch. */
int32_t bake_normals_batched(const bake_asset *assets, int32_t n_assets, const bake_options *opt,
                             void *workspace, size_t workspace_bytes, void *stream);

/* Backward of every asset of the batch (bake_normals_backward semantics per
 * asset, from grad_map into grad_lo_V / grad_hi_N).  Needs the workspace of the
 * last bake_normals_batched with BAKE_FLAG_SAVE on a batch of the same sizes. */
int32_t bake_normals_batched_backward(const bake_asset *assets, int32_t n_assets, void *workspace,
                                      size_t workspace_bytes, void *stream);

/* bake_read_counter for asset `asset` of the last batch that used `workspace`. */
int32_t bake_read_asset_counter(const void *workspace, int32_t asset, int32_t which, void *stream,
                                int64_t *value_out);

/* Traversal autotuner: bakes the batch with every traversal configuration
 * (trav_block x trav_stack x trav_mode = 3 x 3 x 4), `reps` times each,
 * and returns in *best_out the options of `base` (NULL = defaults) with the
 * configuration of the smallest median traversal time; ms_out (NULL or 36
 * floats) receives every configuration's median, in the order block-major,
 * then stack, then mode.  Synchronises the stream; do not record it in a
 * graph.  The outputs of the batch are those of the last configuration run
 * (all configurations give identical results). */
int32_t bake_autotune(const bake_asset *assets, int32_t n_assets, const bake_options *base, int32_t reps,
                      void *workspace, size_t workspace_bytes, void *stream, bake_options *best_out,
                      float *ms_out);

/* ---- mesh simplification (Sec. 6.1) ------------------------------------
 *
 * Quadric-error edge collapse with the edge-constrained optimal placement:
 * every vertex carries the quadric of its faces' planes; collapsing edge
 * (v0, v1) costs min E over the placement under Q = Q_v0 + Q_v1; an interior
 * edge is placed at the solution of A x = -b projected onto the edge
 * (t = <x - v0, v1 - v0> / |v1 - v0|^2 clamped to [0, 1]), at the midpoint
 * when A is singular (det A <= 1e-8 (trace A)^3); boundary vertices stay put
 * and a boundary edge keeps its endpoint of lower error; the same placement
 * ranks and collapses.  A collapse is allowed when the edge has one or two
 * faces, the endpoint rings share exactly that many vertices, the endpoints
 * are not both of three neighbours, an interior edge does not join two
 * boundary vertices, and no face around an endpoint turns its normal to a
 * non-positive dot with the old one.  All of this is FP64.
 *
 * Collapses run in rounds over the whole mesh: edges numbered in (v0, v1)
 * order take the key (float32(cost) bits, number); the eligible edges are the
 * allowed ones with float32 cost at most the k-th smallest, k = ceil(rho *
 * allowed); an eligible edge collapses when its key is the least among the
 * eligible edges at its endpoints and at their neighbours, so the collapses of
 * a round touch disjoint faces; if they would remove more faces than remain
 * above target_faces, only the prefix in key order that fits is applied.  v0
 * (the lower index) survives at the placement with Q_v0 + Q_v1; faces holding
 * both endpoints disappear.  Rounds end when the face count reaches
 * target_faces, when nothing collapses, or after max_rounds.
 *
 * V [n_v,3] f32 and F [n_f,3] i32: device, read only.  Outputs, device and
 * caller-owned: V_out [n_v,3] f32 and F_out [n_f,3] i32 receive the result
 * (the surviving vertices referenced by a face in ascending input index,
 * positions rounded from FP64 to f32; the surviving faces in their input
 * order, renumbered).  HOST outputs: counts_out[2] = (vertices, faces) of the
 * result, *rounds_out = rounds run, stats_out NULL or [max_rounds][4] per
 * round (edges, allowed edges, collapses, faces after the round),
 * times_ms_out NULL or [2]: the summed duration of the per-edge evaluation
 * launches and of the whole call, from HIP events on the stream.
 * flags: BAKE_QEM_MIDPOINT places interior edges at their midpoint (the
 * original placement the section compares against).  Workspace >=
 * bake_qem_workspace_size bytes, 256-byte aligned, overwritten; nothing is
 * allocated.  Unlike the bake, these calls are BLOCKING: the number of rounds
 * depends on the data, so the stream is synchronised once per round to read
 * its counts; they return once the outputs are written.
 * Errors: BAKE_E_INVALID_ARG (NULL pointers, negative counts, target_faces < 4,
 * rho outside (0, 1], max_rounds < 0), BAKE_E_UNSUPPORTED (n_v or n_f >= 2^28),
 * BAKE_E_INDEX (a face with an index outside [0, n_v) or a repeated vertex),
 * BAKE_E_WORKSPACE, BAKE_E_HIP. */
#define BAKE_QEM_MIDPOINT 1u

int32_t bake_qem_workspace_size(int64_t n_v, int64_t n_f, size_t *bytes_out);
int32_t bake_qem_simplify(const float *V, const int32_t *F, int64_t n_v, int64_t n_f, int64_t target_faces,
                          double rho, int32_t max_rounds, uint32_t flags, float *V_out, int32_t *F_out,
                          int64_t *counts_out, int32_t *rounds_out, int64_t *stats_out, float *times_ms_out,
                          void *workspace, size_t workspace_bytes, void *stream);

/* Every edge of the input mesh with its collapse evaluated, as the first
 * round of bake_qem_simplify sees it.  Device outputs (caller-owned, `cap`
 * rows): edges_out [cap][2] i32 (v0 < v1, in (v0, v1) order), valid_out [cap]
 * u8 (the collapse is allowed), faces_out [cap] i32 (faces on the edge; 7
 * stands for seven or more),
 * cost_out [cap] f64 (max(E(p), 0); 0 where no placement was computed),
 * p_out [cap][3] f64 (the placement; zeros where none), Q_out NULL or
 * [n_v][10] f64 (vertex quadrics q00 q01 q02 q03 q11 q12 q13 q22 q23 q33).
 * HOST output *n_edges_out = number of edges; when it exceeds cap nothing is
 * written and the call fails with BAKE_E_INVALID_ARG.  BLOCKING.  Same
 * workspace and errors as bake_qem_simplify. */
int32_t bake_qem_edges(const float *V, const int32_t *F, int64_t n_v, int64_t n_f, uint32_t flags, int64_t cap,
                       int32_t *edges_out, uint8_t *valid_out, int32_t *faces_out, double *cost_out, double *p_out,
                       double *Q_out, int64_t *n_edges_out, void *workspace, size_t workspace_bytes, void *stream);

/* Thread-local message of the last error on this thread ("" if none). */
const char *bake_last_error(void);

/* Library version string. */
const char *bake_version(void);

#ifdef __cplusplus
}
#endif
#endif
