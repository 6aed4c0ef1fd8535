// C ABI of the normal baker: host-side argument validation, workspace carving
// and the stream-ordered launch sequence of the bake (Sec. 6.4):
//   low-poly prep -> UV raster (G-buffer) -> uncovered fill -> LBVH build ->
//   traversal + encode -> dilation -> optional RGB8.
// No device memory is allocated here; all scratch lives in the caller's
// workspace, and nothing synchronises except the explicit query calls.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "../../include/bake.h"
#include "internal.h"

using namespace bake;

namespace {

thread_local char g_err[512] = "";

int32_t fail(int32_t code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int32_t fail(int32_t code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_OR_FAIL(expr)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(BAKE_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

constexpr int64_t kMaxLanes = 256 * 2560;  // upper bound on resident traversal lanes
constexpr int64_t kMaxCount = (int64_t)1 << 30;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Opts {
    int dilate;
    uint32_t flags;
    uint8_t* rgb8;
    TravConfig trav;
};

int32_t parse_opts(const bake_options* o, Opts* out) {
    out->dilate = 2;
    out->flags = 0;
    out->rgb8 = nullptr;
    out->trav.block = 256;
    out->trav.stack = 16;
    out->trav.persist = 0;
    if (!o) return BAKE_OK;
    if (o->dilate_passes < 0 || o->dilate_passes > 64)
        return fail(BAKE_E_INVALID_ARG, "dilate_passes %d outside [0, 64]", o->dilate_passes);
    out->dilate = o->dilate_passes;
    if (o->flags & ~(uint32_t)(BAKE_FLAG_SAVE | BAKE_FLAG_TIMING | BAKE_FLAG_COUNT))
        return fail(BAKE_E_INVALID_ARG, "unknown flag bits 0x%x", o->flags);
    out->flags = o->flags;
    out->rgb8 = o->out_rgb8;
    if (o->trav_block != 0) {
        if (o->trav_block != 64 && o->trav_block != 128 && o->trav_block != 256)
            return fail(BAKE_E_INVALID_ARG, "trav_block %d not in {64,128,256}", o->trav_block);
        out->trav.block = o->trav_block;
    }
    if (o->trav_stack != 0) {
        if (o->trav_stack != 8 && o->trav_stack != 16 && o->trav_stack != 32)
            return fail(BAKE_E_INVALID_ARG, "trav_stack %d not in {8,16,32}", o->trav_stack);
        out->trav.stack = o->trav_stack;
    }
    if (o->trav_persist < -1 || o->trav_persist > 1)
        return fail(BAKE_E_INVALID_ARG, "trav_persist %d not in {-1,0,1}", o->trav_persist);
    if (o->trav_persist >= 0) out->trav.persist = o->trav_persist;
    return BAKE_OK;
}

int32_t check_sizes(int64_t nhv, int64_t nhf, int64_t nlv, int64_t nlf, int32_t res) {
    if (nhv < 0 || nhf < 0 || nlv < 0 || nlf < 0)
        return fail(BAKE_E_INVALID_ARG, "negative count");
    if (nhv >= kMaxCount || nhf >= kMaxCount || nlv >= kMaxCount || nlf >= kMaxCount)
        return fail(BAKE_E_UNSUPPORTED, "counts must be < 2^30");
    if (nhf > 0 && nhv == 0) return fail(BAKE_E_INVALID_ARG, "hi triangles without hi vertices");
    if (nlf > 0 && nlv == 0) return fail(BAKE_E_INVALID_ARG, "lo triangles without lo vertices");
    if (res < 1 || res > 16384 || (res & (res - 1)) != 0)
        return fail(BAKE_E_UNSUPPORTED, "res %d must be a power of two in [1, 16384]", res);
    return BAKE_OK;
}

Layout make_layout(int64_t nhv, int64_t nhf, int64_t nlv, int64_t nlf, int32_t res, uint32_t flags) {
    (void)nhv;
    Layout L;
    memset(&L, 0, sizeof L);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.n_texels = (int64_t)res * res;
    L.max_rays = L.n_texels;
    L.sort_blocks = (nhf + 4095) / 4096;
    int64_t scan_n = std::max<int64_t>(std::max<int64_t>(nlv, nlf), 256 * L.sort_blocks);
    if (flags & BAKE_FLAG_SAVE) scan_n = std::max<int64_t>(scan_n, radix_hist_elems(3 * L.max_rays));
    L.scan_tmp_n = scan_tmp_elems(scan_n) + 1;
    int64_t lanes = std::min<int64_t>(std::max<int64_t>(L.max_rays, 256), kMaxLanes);
    L.spill_lanes = (lanes + 255) / 256 * 256;

    L.status = take(4);
    L.counters = take(4 * kCntSlots);
    L.lo_n = take(16 * (size_t)nlv);
    L.lo_deg = take(4 * (size_t)nlv);
    L.lo_off = take(4 * (size_t)(nlv + 1));
    L.lo_cur = take(4 * (size_t)nlv);
    L.lo_adj = take(12 * (size_t)nlf);
    L.face_t = take(16 * (size_t)nlf);
    L.face_uv = take(32 * (size_t)nlf);
    L.face_cnt = take(4 * (size_t)nlf);
    L.face_off = take(4 * (size_t)(nlf + 1));
    L.scan_tmp = take(4 * (size_t)L.scan_tmp_n);
    L.facemap = take(4 * (size_t)L.n_texels);
    L.level = take((size_t)L.n_texels);
    L.rays = take(16 * (size_t)L.max_rays);
    L.hits = (flags & BAKE_FLAG_SAVE) ? take(16 * (size_t)L.max_rays) : off;
    L.bounds_part = take(4 * 6 * 512);
    L.bounds = take(4 * 6);
    L.keys0 = take(4 * (size_t)nhf);
    L.vals0 = take(4 * (size_t)nhf);
    L.keys1 = take(4 * (size_t)nhf);
    L.vals1 = take(4 * (size_t)nhf);
    L.hist = take(4 * 256 * (size_t)L.sort_blocks);
    L.nodes = take(64 * (size_t)std::max<int64_t>(nhf - 1, 1));
    L.leaves = take(48 * (size_t)std::max<int64_t>(nhf, 1));
    L.node_parent = take(4 * (size_t)std::max<int64_t>(nhf - 1, 1));
    L.leaf_parent = take(4 * (size_t)std::max<int64_t>(nhf, 1));
    L.refit_cnt = take(4 * (size_t)std::max<int64_t>(nhf - 1, 1));
    L.node_range = take(8 * (size_t)std::max<int64_t>(nhf - 1, 1));
    L.frontier = take(4 * (size_t)treelet_cap(nhf));
    L.treelets = take(16 * (size_t)treelet_cap(nhf));
    L.spill = take(4 * (size_t)kMaxDepth * (size_t)L.spill_lanes);
    if (flags & BAKE_FLAG_SAVE) {
        const size_t items = 3 * (size_t)L.max_rays;
        L.bwd_ray = take(48 * (size_t)L.max_rays);
        L.bwd_k0 = take(4 * items);
        L.bwd_v0 = take(4 * items);
        L.bwd_k1 = take(4 * items);
        L.bwd_v1 = take(4 * items);
        L.bwd_hist = take(4 * (size_t)radix_hist_elems((int64_t)items));
        L.bwd_face1 = take(72 * (size_t)nlf);
        L.bwd_face2 = take(36 * (size_t)nlf);
        L.bwd_sbar = take(12 * (size_t)nlv);
        L.bwd_vbar = take(12 * (size_t)nlv);
    }
    L.total = off;
    return L;
}

// ---- forwards that saved their state (for the backward pass) ---------------
// Host-side record of the last saved forwards, keyed by workspace, so a
// backward call can check it matches a saved forward of the same sizes.  It
// is process-wide (autograd may run the backward on another thread).
struct Saved {
    const void* ws;
    int64_t nhv, nhf, nlv, nlf;
    int32_t res;
};
constexpr int kSavedSlots = 64;
std::mutex g_saved_mu;
Saved g_saved[kSavedSlots];
int g_saved_next = 0;

void remember_saved(const void* ws, int64_t nhv, int64_t nhf, int64_t nlv, int64_t nlf, int32_t res) {
    std::lock_guard<std::mutex> lk(g_saved_mu);
    for (int i = 0; i < kSavedSlots; ++i)
        if (g_saved[i].ws == ws) {
            g_saved[i] = Saved{ws, nhv, nhf, nlv, nlf, res};
            return;
        }
    g_saved[g_saved_next] = Saved{ws, nhv, nhf, nlv, nlf, res};
    g_saved_next = (g_saved_next + 1) % kSavedSlots;
}

void forget_saved(const void* ws) {
    std::lock_guard<std::mutex> lk(g_saved_mu);
    for (int i = 0; i < kSavedSlots; ++i)
        if (g_saved[i].ws == ws) g_saved[i].ws = nullptr;
}

bool was_saved(const void* ws, int64_t nhv, int64_t nhf, int64_t nlv, int64_t nlf, int32_t res) {
    std::lock_guard<std::mutex> lk(g_saved_mu);
    for (int i = 0; i < kSavedSlots; ++i) {
        const Saved& v = g_saved[i];
        if (v.ws == ws && ws != nullptr)
            return v.nhv == nhv && v.nhf == nhf && v.nlv == nlv && v.nlf == nlf && v.res == res;
    }
    return false;
}

// ---- per-thread stage timing ---------------------------------------------
// A ring of event sets, so the stage times of many consecutive bakes can be
// read back after they ran, without synchronising between them.
constexpr int kStages = 6;
constexpr int kRing = 64;
struct Timing {
    hipEvent_t ev[kRing][kStages];
    bool created = false;
    int next = 0;   // ring slot of the next timed bake
    int count = 0;  // timed bakes recorded (saturates at kRing)
};
thread_local Timing g_tim;

hipError_t tim_record(bool on, int k, hipStream_t s) {
    if (!on) return hipSuccess;
    if (!g_tim.created) {
        for (int r = 0; r < kRing; ++r)
            for (int i = 0; i < kStages; ++i) {
                hipError_t e = hipEventCreate(&g_tim.ev[r][i]);
                if (e != hipSuccess) return e;
            }
        g_tim.created = true;
    }
    return hipEventRecord(g_tim.ev[g_tim.next][k], s);
}

void tim_commit(bool on) {
    if (!on) return;
    g_tim.next = (g_tim.next + 1) % kRing;
    if (g_tim.count < kRing) ++g_tim.count;
}

// Stage times of ring slot r: 0 lo prep, 1 raster, 2 BVH, 3 traversal, 4 dilation, 5 total.
int32_t slot_times(int r, float* ms) {
    HIP_OR_FAIL(hipEventSynchronize(g_tim.ev[r][kStages - 1]));
    for (int k = 0; k < kStages; ++k) {
        float v = 0.f;
        if (k < kStages - 1) {
            HIP_OR_FAIL(hipEventElapsedTime(&v, g_tim.ev[r][k], g_tim.ev[r][k + 1]));
        } else {
            HIP_OR_FAIL(hipEventElapsedTime(&v, g_tim.ev[r][0], g_tim.ev[r][kStages - 1]));
        }
        ms[k] = v;
    }
    return BAKE_OK;
}

int32_t validate_common(const float* hi_V, int64_t nhv, const int32_t* hi_F, int64_t nhf,
                        const float* hi_N, const float* lo_V, int64_t nlv, const int32_t* lo_F,
                        int64_t nlf, const float* lo_UV, int32_t res, float max_dist) {
    int32_t rc = check_sizes(nhv, nhf, nlv, nlf, res);
    if (rc) return rc;
    if (nhv > 0 && (!hi_V || !hi_N)) return fail(BAKE_E_INVALID_ARG, "hi_V / hi_N is NULL");
    if (nhf > 0 && !hi_F) return fail(BAKE_E_INVALID_ARG, "hi_F is NULL");
    if (nlv > 0 && !lo_V) return fail(BAKE_E_INVALID_ARG, "lo_V is NULL");
    if (nlf > 0 && (!lo_F || !lo_UV)) return fail(BAKE_E_INVALID_ARG, "lo_F / lo_UV is NULL");
    if (!(max_dist > 0.f) || !(max_dist < INFINITY))
        return fail(BAKE_E_INVALID_ARG, "max_dist must be finite and > 0");
    return BAKE_OK;
}

int32_t check_workspace(const void* ws, size_t bytes, const Layout& L) {
    if (!ws) return fail(BAKE_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(BAKE_E_WORKSPACE, "workspace not 256-byte aligned");
    if (bytes < L.total)
        return fail(BAKE_E_WORKSPACE, "workspace has %zu bytes, needs %zu", bytes, L.total);
    return BAKE_OK;
}

}  // namespace

extern "C" {

void bake_default_options(bake_options* opt) {
    if (!opt) return;
    memset(opt, 0, sizeof *opt);
    opt->dilate_passes = 2;
    opt->trav_persist = -1;
}

const char* bake_last_error(void) { return g_err; }

const char* bake_version(void) { return "paper_2605_26137_amd bake 0.1 (gfx950)"; }

int32_t bake_workspace_size(int64_t n_hi_v, int64_t n_hi_f, int64_t n_lo_v, int64_t n_lo_f,
                            int32_t res, const bake_options* opt, size_t* bytes_out) {
    g_err[0] = 0;
    if (!bytes_out) return fail(BAKE_E_INVALID_ARG, "bytes_out is NULL");
    Opts o;
    int32_t rc = parse_opts(opt, &o);
    if (rc) return rc;
    if ((rc = check_sizes(n_hi_v, n_hi_f, n_lo_v, n_lo_f, res))) return rc;
    *bytes_out = make_layout(n_hi_v, n_hi_f, n_lo_v, n_lo_f, res, o.flags).total;
    return BAKE_OK;
}

int32_t bake_workspace_view(int64_t n_hi_v, int64_t n_hi_f, int64_t n_lo_v, int64_t n_lo_f,
                            int32_t res, const bake_options* opt, int32_t which,
                            size_t* offset_out, size_t* bytes_out) {
    g_err[0] = 0;
    if (!offset_out || !bytes_out) return fail(BAKE_E_INVALID_ARG, "NULL output");
    Opts o;
    int32_t rc = parse_opts(opt, &o);
    if (rc) return rc;
    if ((rc = check_sizes(n_hi_v, n_hi_f, n_lo_v, n_lo_f, res))) return rc;
    Layout L = make_layout(n_hi_v, n_hi_f, n_lo_v, n_lo_f, res, o.flags);
    switch (which) {
        case BAKE_VIEW_RAYS: *offset_out = L.rays; *bytes_out = 16 * (size_t)L.max_rays; break;
        case BAKE_VIEW_HITS:
            if (!(o.flags & BAKE_FLAG_SAVE)) return fail(BAKE_E_INVALID_ARG, "hits need BAKE_FLAG_SAVE");
            *offset_out = L.hits; *bytes_out = 16 * (size_t)L.max_rays; break;
        case BAKE_VIEW_FACEMAP: *offset_out = L.facemap; *bytes_out = 4 * (size_t)L.n_texels; break;
        case BAKE_VIEW_LO_N: *offset_out = L.lo_n; *bytes_out = 16 * (size_t)n_lo_v; break;
        case BAKE_VIEW_SORTED: *offset_out = L.keys0; *bytes_out = 8 * (size_t)n_hi_f; break;
        case BAKE_VIEW_NODES:
            *offset_out = L.nodes; *bytes_out = 64 * (size_t)std::max<int64_t>(n_hi_f - 1, 0); break;
        case BAKE_VIEW_LEAVES: *offset_out = L.leaves; *bytes_out = 48 * (size_t)n_hi_f; break;
        case BAKE_VIEW_FACE_T: *offset_out = L.face_t; *bytes_out = 16 * (size_t)n_lo_f; break;
        default: return fail(BAKE_E_INVALID_ARG, "unknown view %d", which);
    }
    return BAKE_OK;
}

int32_t bake_normals(const float* hi_V, int64_t n_hi_v, const int32_t* hi_F, int64_t n_hi_f,
                     const float* hi_N, const float* lo_V, int64_t n_lo_v, const int32_t* lo_F,
                     int64_t n_lo_f, const float* lo_UV, int32_t res, float max_dist,
                     float* out_map, int32_t* out_hit, const bake_options* opt, void* workspace,
                     size_t workspace_bytes, void* stream) {
    g_err[0] = 0;
    Opts o;
    int32_t rc = parse_opts(opt, &o);
    if (rc) return rc;
    if ((rc = validate_common(hi_V, n_hi_v, hi_F, n_hi_f, hi_N, lo_V, n_lo_v, lo_F, n_lo_f, lo_UV,
                              res, max_dist)))
        return rc;
    if (!out_map || !out_hit) return fail(BAKE_E_INVALID_ARG, "out_map / out_hit is NULL");
    Layout L = make_layout(n_hi_v, n_hi_f, n_lo_v, n_lo_f, res, o.flags);
    if ((rc = check_workspace(workspace, workspace_bytes, L))) return rc;
    // the save order of the ray list must be pinned for the backward pass, and
    // the output buffers must not overlap the workspace
    char* ws = (char*)workspace;
    hipStream_t s = (hipStream_t)stream;
    const bool tim = (o.flags & BAKE_FLAG_TIMING) != 0;

    HIP_OR_FAIL(tim_record(tim, 0, s));
    HIP_OR_FAIL(fill_u32((uint32_t*)(ws + L.status), 0, 1, s));
    HIP_OR_FAIL(fill_u32((uint32_t*)(ws + L.counters), 0, kCntSlots, s));
    HIP_OR_FAIL(launch_lo_prep(lo_V, n_lo_v, lo_F, n_lo_f, lo_UV, res, L, ws, s));
    HIP_OR_FAIL(tim_record(tim, 1, s));
    HIP_OR_FAIL(launch_raster(n_lo_f, res, L, ws, s));
    HIP_OR_FAIL(launch_fill_uncovered(res, out_map, out_hit, L, ws, s));
    HIP_OR_FAIL(tim_record(tim, 2, s));
    HIP_OR_FAIL(launch_bvh_build(hi_V, n_hi_v, hi_F, n_hi_f, L, ws, s));
    HIP_OR_FAIL(tim_record(tim, 3, s));
    TravConfig tc = o.trav;
    tc.count = (o.flags & BAKE_FLAG_COUNT) != 0;
    HIP_OR_FAIL(launch_traverse(lo_V, lo_F, n_lo_f, hi_F, n_hi_v, n_hi_f, hi_N, max_dist, out_map,
                                out_hit, (o.flags & BAKE_FLAG_SAVE) != 0, tc, L, ws, s));
    HIP_OR_FAIL(tim_record(tim, 4, s));
    HIP_OR_FAIL(launch_dilate(res, o.dilate, out_map, L, ws, s));
    if (o.rgb8) HIP_OR_FAIL(launch_rgb8(res, out_map, o.rgb8, s));
    HIP_OR_FAIL(tim_record(tim, 5, s));
    tim_commit(tim);
    if (o.flags & BAKE_FLAG_SAVE) remember_saved(workspace, n_hi_v, n_hi_f, n_lo_v, n_lo_f, res);
    else forget_saved(workspace);
    return BAKE_OK;
}

int32_t bake_normals_backward(const float* hi_V, int64_t n_hi_v, const int32_t* hi_F,
                              int64_t n_hi_f, const float* hi_N, const float* lo_V, int64_t n_lo_v,
                              const int32_t* lo_F, int64_t n_lo_f, const float* lo_UV, int32_t res,
                              float max_dist, const float* grad_map, float* grad_lo_V,
                              float* grad_hi_N, void* workspace, size_t workspace_bytes,
                              void* stream) {
    g_err[0] = 0;
    int32_t rc = validate_common(hi_V, n_hi_v, hi_F, n_hi_f, hi_N, lo_V, n_lo_v, lo_F, n_lo_f, lo_UV,
                                 res, max_dist);
    if (rc) return rc;
    if (!grad_map) return fail(BAKE_E_INVALID_ARG, "grad_map is NULL");
    Layout L = make_layout(n_hi_v, n_hi_f, n_lo_v, n_lo_f, res, BAKE_FLAG_SAVE);
    if ((rc = check_workspace(workspace, workspace_bytes, L))) return rc;
    if (!was_saved(workspace, n_hi_v, n_hi_f, n_lo_v, n_lo_f, res))
        return fail(BAKE_E_STATE,
                    "no forward bake with BAKE_FLAG_SAVE and these sizes used this workspace");
    if (!grad_lo_V && !grad_hi_N) return BAKE_OK;
    HIP_OR_FAIL(launch_backward(hi_V, hi_F, n_hi_v, hi_N, lo_V, lo_F, n_lo_v, n_lo_f, grad_map, grad_lo_V,
                                grad_hi_N, L, (char*)workspace, (hipStream_t)stream));
    return BAKE_OK;
}

int32_t bake_sq_loss(const float* map, const float* target, int64_t n, float* grad_out, float* loss_out,
                     void* scratch, size_t scratch_bytes, void* stream) {
    g_err[0] = 0;
    if (n < 0) return fail(BAKE_E_INVALID_ARG, "negative count");
    if ((n > 0 && (!map || !target)) || !loss_out) return fail(BAKE_E_INVALID_ARG, "NULL argument");
    const size_t need = 4 * (size_t)((n + 255) / 256 + 1);
    if (!scratch || scratch_bytes < need)
        return fail(BAKE_E_WORKSPACE, "scratch has %zu bytes, needs %zu", scratch_bytes, need);
    HIP_OR_FAIL(launch_sq_loss(map, target, n, grad_out, loss_out, (float*)scratch, (hipStream_t)stream));
    return BAKE_OK;
}

int32_t bake_query_status(const void* workspace, void* stream, uint32_t* status_out) {
    g_err[0] = 0;
    if (!workspace || !status_out) return fail(BAKE_E_INVALID_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    uint32_t v = 0;
    HIP_OR_FAIL(hipMemcpyAsync(&v, workspace, 4, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    *status_out = v;
    return BAKE_OK;
}

int32_t bake_read_counter(const void* workspace, int32_t which, void* stream, int64_t* value_out) {
    g_err[0] = 0;
    if (!workspace || !value_out) return fail(BAKE_E_INVALID_ARG, "NULL argument");
    if (which < 0 || which > 2) return fail(BAKE_E_INVALID_ARG, "unknown counter %d", which);
    hipStream_t s = (hipStream_t)stream;
    uint32_t v[kCntSlots];
    // counters sit right after the 256-byte status block
    HIP_OR_FAIL(hipMemcpyAsync(v, (const char*)workspace + 256, sizeof v, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    if (which == 0) *value_out = v[kCntRays];
    else if (which == 1) *value_out = (int64_t)v[kCntBoxLo] | ((int64_t)v[kCntBoxLo + 1] << 32);
    else *value_out = (int64_t)v[kCntTriLo] | ((int64_t)v[kCntTriLo + 1] << 32);
    return BAKE_OK;
}

int32_t bake_stage_times(float* ms_out, int32_t n) {
    g_err[0] = 0;
    if (!ms_out || n < 0) return fail(BAKE_E_INVALID_ARG, "bad output");
    if (g_tim.count == 0) return fail(BAKE_E_STATE, "no timed bake on this thread");
    float ms[kStages];
    int32_t rc = slot_times((g_tim.next + kRing - 1) % kRing, ms);
    if (rc) return rc;
    int m = std::min<int>(n, kStages);
    for (int k = 0; k < m; ++k) ms_out[k] = ms[k];
    return m;
}

int32_t bake_stage_history(float* ms_out, int32_t max_bakes) {
    g_err[0] = 0;
    if (!ms_out || max_bakes < 0) return fail(BAKE_E_INVALID_ARG, "bad output");
    int m = std::min<int>(max_bakes, g_tim.count);
    for (int i = 0; i < m; ++i) {
        int r = (g_tim.next + kRing - m + i) % kRing;  // oldest first
        int32_t rc = slot_times(r, ms_out + (size_t)i * kStages);
        if (rc) return rc;
    }
    return m;
}

}  // extern "C"
