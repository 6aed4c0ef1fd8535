// C ABI of the normal baker: host-side argument validation, the batch plan
// (asset table, per-grid block prefix tables, workspace carving) and the
// stream-ordered launch sequence of the bake (Sec. 6.4):
//   low-poly prep -> UV raster (G-buffer) -> uncovered fill -> LBVH build ->
//   traversal + encode -> dilation -> optional RGB8,
// and of its backward.  A single bake is a batch of one asset.  No device
// memory is allocated here; all scratch lives in the caller's workspace, the
// asset table reaches the device as kernel arguments, and nothing
// synchronises except the explicit query, timing and tuning calls.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

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
constexpr int kMaxAssets = 65536;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

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
    out->trav.mode = 3;
    if (!o) return BAKE_OK;
    if (o->dilate_passes < 0 || o->dilate_passes > 64)
        return fail(BAKE_E_INVALID_ARG, "dilate_passes %d outside [0, 64]", o->dilate_passes);
    out->dilate = o->dilate_passes;
    if (o->flags & ~(uint32_t)(BAKE_FLAG_SAVE | BAKE_FLAG_TIMING | BAKE_FLAG_COUNT | BAKE_FLAG_ONE_STREAM |
                               BAKE_FLAG_ONE_QUEUE))
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
    if (o->trav_mode < -1 || o->trav_mode > 3)
        return fail(BAKE_E_INVALID_ARG, "trav_mode %d not in {-1,0,1,2,3}", o->trav_mode);
    if (o->trav_mode >= 0) out->trav.mode = o->trav_mode;
    if (o->query != BAKE_QUERY_RAY && o->query != BAKE_QUERY_CLOSEST)
        return fail(BAKE_E_INVALID_ARG, "query %d unknown", o->query);
    out->trav.closest = o->query == BAKE_QUERY_CLOSEST;
    if (out->trav.closest && (o->flags & BAKE_FLAG_SAVE))
        return fail(BAKE_E_UNSUPPORTED, "the closest-point query has no backward (BAKE_FLAG_SAVE)");
    return BAKE_OK;
}

struct Sizes {
    int64_t nhv, nhf, nlv, nlf;
    int32_t res;
};

int32_t check_sizes(const Sizes& z) {
    if (z.nhv < 0 || z.nhf < 0 || z.nlv < 0 || z.nlf < 0)
        return fail(BAKE_E_INVALID_ARG, "negative count");
    if (z.nhv >= kMaxCount || z.nhf >= kMaxCount || z.nlv >= kMaxCount || z.nlf >= kMaxCount)
        return fail(BAKE_E_UNSUPPORTED, "counts must be < 2^30");
    if (z.nhf > 0 && z.nhv == 0) return fail(BAKE_E_INVALID_ARG, "hi triangles without hi vertices");
    if (z.nlf > 0 && z.nlv == 0) return fail(BAKE_E_INVALID_ARG, "lo triangles without lo vertices");
    if (z.res < 1 || z.res > 16384 || (z.res & (z.res - 1)) != 0)
        return fail(BAKE_E_UNSUPPORTED, "res %d must be a power of two in [1, 16384]", z.res);
    return BAKE_OK;
}

// Blocks of grid g for one asset.
int64_t grid_blocks(int g, const Sizes& z) {
    const int64_t tex = (int64_t)z.res * z.res;
    switch (g) {
        case kGLoF: return cdiv(z.nlf, 256);
        case kGLoFWave: return cdiv(z.nlf, 4);
        case kGLoV: return cdiv(z.nlv, 256);
        case kGHiV: return cdiv(z.nhv, 256);
        case kGHiF: return cdiv(z.nhf, 256);
        case kGSort: return cdiv(z.nhf, kSortTile);
        case kGTex: return cdiv(tex, 256);
        case kGTex3: return cdiv(3 * tex, 256);
        case kGBwdSort: return cdiv(3 * tex, kSortTile);
        case kGTile: return cdiv(z.res, kFinishTile) * cdiv(z.res, kFinishTile);
    }
    return 0;
}

// The batch plan: asset table (pointers filled by the caller), grid prefix
// tables and the workspace layout.
struct Plan {
    Layout L;
    std::vector<AssetDev> A;
    std::vector<AssetGrad> G;
    std::vector<int32_t> gpf;  // [kGridCount][n + 1]
    uint64_t sig = 0;          // signature of the batch's sizes
};

int32_t make_plan(const Sizes* z, int n, uint32_t flags, Plan* P) {
    if (n < 1 || n > kMaxAssets) return fail(BAKE_E_INVALID_ARG, "n_assets %d outside [1, %d]", n, kMaxAssets);
    Layout& L = P->L;
    memset(&L, 0, sizeof L);
    L.n = n;
    L.save = (flags & BAKE_FLAG_SAVE) != 0;
    P->A.assign(n, AssetDev{});
    P->gpf.assign((size_t)kGridCount * (n + 1), 0);
    uint64_t sig = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { sig = (sig ^ v) * 1099511628211ull; };
    mix((uint64_t)n);
    int64_t gsum[kGridCount] = {};
    int64_t max_hv = 0;
    for (int a = 0; a < n; ++a) {
        int32_t rc = check_sizes(z[a]);
        if (rc) return rc;
        AssetDev& d = P->A[a];
        d.nhv = (int32_t)z[a].nhv;
        d.nhf = (int32_t)z[a].nhf;
        d.nlv = (int32_t)z[a].nlv;
        d.nlf = (int32_t)z[a].nlf;
        d.res = z[a].res;
        d.log2res = 0;
        while ((1 << d.log2res) < d.res) ++d.log2res;
        d.index = a;
        d.lv = L.t_lv;
        d.lf = L.t_lf;
        d.hf = L.t_hf;
        d.node = L.t_node;
        d.tex = L.t_tex;
        d.stile = L.t_stile;
        d.btile = L.t_btile;
        d.tl = L.t_tl;
        const int64_t tex = (int64_t)z[a].res * z[a].res;
        L.t_lv += z[a].nlv;
        L.t_lf += z[a].nlf;
        L.t_hv += z[a].nhv;
        L.t_hf += z[a].nhf;
        L.t_node += std::max<int64_t>(z[a].nhf - 1, 0);
        L.t_tex += tex;
        L.t_stile += cdiv(z[a].nhf, kSortTile);
        L.t_btile += cdiv(3 * tex, kSortTile);
        L.t_tl += treelet_cap(z[a].nhf);
        max_hv = std::max(max_hv, z[a].nhv);
        for (int g = 0; g < kGridCount; ++g) {
            P->gpf[(size_t)g * (n + 1) + a] = (int32_t)gsum[g];
            gsum[g] += grid_blocks(g, z[a]);
        }
        mix((uint64_t)z[a].nhv);
        mix((uint64_t)z[a].nhf);
        mix((uint64_t)z[a].nlv);
        mix((uint64_t)z[a].nlf);
        mix((uint64_t)z[a].res);
    }
    for (int g = 0; g < kGridCount; ++g) {
        if (gsum[g] >= ((int64_t)1 << 31)) return fail(BAKE_E_UNSUPPORTED, "batch too large (grid %d)", g);
        P->gpf[(size_t)g * (n + 1) + n] = (int32_t)gsum[g];
    }
    if (L.t_hf >= ((int64_t)1 << 31) || 3 * L.t_tex >= ((int64_t)1 << 32) || L.t_lv >= ((int64_t)1 << 31) ||
        L.t_lf >= ((int64_t)1 << 31))
        return fail(BAKE_E_UNSUPPORTED, "batch too large: needs sum(n_hi_f) < 2^31 and 3 sum(res^2) < 2^32");
    L.max_hv_bits = 1;
    while (L.max_hv_bits < 32 && ((int64_t)1 << L.max_hv_bits) <= max_hv) ++L.max_hv_bits;  // keys in [0, nhv]
    P->sig = sig ^ (L.save ? 0x5A5Aull : 0ull);

    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    const int64_t scan_n = std::max<int64_t>(L.t_lv, L.t_lf);  // the low-poly CSR and raster scans
    L.scan_tmp_n = scan_tmp_elems(scan_n) + 1;
    int64_t lanes = std::min<int64_t>(std::max<int64_t>(L.t_tex, 256), kMaxLanes);
    L.spill_lanes = (lanes + 255) / 256 * 256;

    L.status = take(4);  // the status block is 256 bytes: counters start at 256
    L.counters = take(4 * (size_t)kCntSlots * n);
    L.gcnt = take(4 * (size_t)kGcSlots);
    // the BVH sort's super-tile rows: zeroed with the counters before the table
    L.sup = take(4 * 256 * (size_t)kSortPasses * (size_t)sort_super_rows(L.t_stile, n));
    L.table = take(sizeof(AssetDev) * (size_t)n + 4 * (size_t)kGridCount * (n + 1));
    L.gpf = L.table + sizeof(AssetDev) * (size_t)n;
    L.grads = take(sizeof(AssetGrad) * (size_t)n);
    L.ray_pf = take(4 * (size_t)(n + 1));
    L.rb_pf = take(4 * (size_t)(n + 1));
    L.tl_pf = take(4 * (size_t)(n + 1));
    L.bt_pf = take(4 * (size_t)(n + 1));
    L.lo_n = take(16 * (size_t)L.t_lv);
    L.lo_deg = take(4 * (size_t)L.t_lv);
    L.lo_off = take(4 * (size_t)(L.t_lv + 1));
    L.lo_cur = take(4 * (size_t)L.t_lv);
    L.lo_adj = take(12 * (size_t)L.t_lf);
    L.face_t = take(16 * (size_t)L.t_lf);
    L.face_uv = take(32 * (size_t)L.t_lf);
    L.face_cnt = take(4 * (size_t)L.t_lf);
    L.face_off = take(4 * (size_t)(L.t_lf + 1));
    L.scan_tmp = take(4 * (size_t)L.scan_tmp_n);
    L.facemap = take(4 * (size_t)L.t_tex);
    L.level = take((size_t)L.t_tex);
    L.rays = take(16 * (size_t)L.t_tex);
    L.hits = L.save ? take(16 * (size_t)L.t_tex) : off;
    L.bounds_part = take(24 * (size_t)kBoundsSplit * (size_t)L.t_stile);
    L.bounds = take(24 * (size_t)n);
    L.keys0 = take(4 * (size_t)L.t_hf);
    L.vals0 = take(4 * (size_t)L.t_hf);
    L.keys1 = take(4 * (size_t)L.t_hf);
    L.vals1 = take(4 * (size_t)L.t_hf);
    L.hist = take(4 * 256 * (size_t)L.t_stile);
    L.nodes = take(64 * (size_t)L.t_node);
    L.nodes_c = take(32 * (size_t)L.t_node);
    L.leaves = take(48 * (size_t)L.t_hf);
    L.node_parent = take(4 * (size_t)L.t_node);
    L.leaf_parent = take(4 * (size_t)L.t_hf);
    L.refit_cnt = take(4 * (size_t)L.t_node);
    L.frontier = take(4 * (size_t)L.t_tl);
    L.treelets = take(16 * (size_t)L.t_tl);
    L.top = take(8 * (size_t)L.t_tl);
    L.child = take(4 * (size_t)L.t_node);
    L.spill = take(4 * (size_t)kMaxDepth * (size_t)L.spill_lanes);
    if (L.save) {
        const size_t items = 3 * (size_t)L.t_tex;
        L.bwd_ray = take(36 * (size_t)L.t_tex);
        L.bwd_hterm = take(32 * (size_t)L.t_tex);
        L.bwd_k0 = take(4 * items);
        L.bwd_v0 = take(4 * items);
        L.bwd_k1 = take(4 * items);
        L.bwd_v1 = take(4 * items);
        L.bwd_hist = take(4 * 256 * (size_t)L.t_btile);
        L.bwd_sup = take(4 * 256 * (size_t)kSortPasses * (size_t)sort_super_rows(L.t_btile, n));
        L.bwd_face1 = take(72 * (size_t)L.t_lf);
        L.bwd_face2 = take(36 * (size_t)L.t_lf);
        L.bwd_sbar = take(12 * (size_t)L.t_lv);
        L.bwd_vbar = take(12 * (size_t)L.t_lv);
    }
    L.total = off;
    return BAKE_OK;
}

Sizes sizes_of(const bake_asset& a) { return Sizes{a.n_hi_v, a.n_hi_f, a.n_lo_v, a.n_lo_f, a.res}; }

int32_t plan_batch(const bake_asset* as, int32_t n, uint32_t flags, Plan* P) {
    if (!as) return fail(BAKE_E_INVALID_ARG, "assets is NULL");
    if (n < 1 || n > kMaxAssets) return fail(BAKE_E_INVALID_ARG, "n_assets %d outside [1, %d]", n, kMaxAssets);
    std::vector<Sizes> z(n);
    for (int a = 0; a < n; ++a) z[a] = sizes_of(as[a]);
    return make_plan(z.data(), n, flags, P);
}

int32_t validate_asset(const bake_asset& a, int idx) {
    if (a.n_hi_v > 0 && (!a.hi_V || !a.hi_N))
        return fail(BAKE_E_INVALID_ARG, "asset %d: hi_V / hi_N is NULL", idx);
    if (a.n_hi_f > 0 && !a.hi_F) return fail(BAKE_E_INVALID_ARG, "asset %d: hi_F is NULL", idx);
    if (a.n_lo_v > 0 && !a.lo_V) return fail(BAKE_E_INVALID_ARG, "asset %d: lo_V is NULL", idx);
    if (a.n_lo_f > 0 && (!a.lo_F || !a.lo_UV))
        return fail(BAKE_E_INVALID_ARG, "asset %d: lo_F / lo_UV is NULL", idx);
    if (!(a.max_dist > 0.f) || !(a.max_dist < INFINITY))
        return fail(BAKE_E_INVALID_ARG, "asset %d: max_dist must be finite and > 0", idx);
    return BAKE_OK;
}

void fill_pointers(const bake_asset* as, Plan* P) {
    for (int a = 0; a < P->L.n; ++a) {
        AssetDev& d = P->A[a];
        d.hi_V = as[a].hi_V;
        d.hi_F = as[a].hi_F;
        d.hi_N = as[a].hi_N;
        d.lo_V = as[a].lo_V;
        d.lo_F = as[a].lo_F;
        d.lo_UV = as[a].lo_UV;
        d.out_map = as[a].out_map;
        d.out_hit = as[a].out_hit;
        d.out_rgb8 = as[a].out_rgb8;
        d.max_dist = as[a].max_dist;
    }
    P->G.assign(P->L.n, AssetGrad{});
    for (int a = 0; a < P->L.n; ++a) P->G[a] = AssetGrad{as[a].grad_map, as[a].grad_lo_V, as[a].grad_hi_N};
}

BatchHost host_view(const Plan& P, char* ws) {
    BatchHost H;
    H.L = P.L;
    H.A = P.A.data();
    H.gpf = P.gpf.data();
    H.ws = ws;
    const Layout& L = P.L;
    H.dev.A = (const AssetDev*)(ws + L.table);
    H.dev.G = (const AssetGrad*)(ws + L.grads);
    H.dev.gpf = (const int32_t*)(ws + L.gpf);
    H.dev.ray_pf = (const uint32_t*)(ws + L.ray_pf);
    H.dev.rb_pf = (const uint32_t*)(ws + L.rb_pf);
    H.dev.tl_pf = (const uint32_t*)(ws + L.tl_pf);
    H.dev.bt_pf = (const uint32_t*)(ws + L.bt_pf);
    H.dev.cnt = (uint32_t*)(ws + L.counters);
    H.dev.gcnt = (uint32_t*)(ws + L.gcnt);
    H.dev.status = (uint32_t*)(ws + L.status);
    H.dev.n = L.n;
    H.dev.seal = 0;
    return H;
}

// ---- forwards that saved their state (for the backward pass) ---------------
// Process-wide record of the last saved forwards, keyed by workspace, so a
// backward call can check it matches a saved forward of the same batch sizes
// (autograd may run the backward on another thread).
struct Saved {
    const void* ws;
    uint64_t sig;
    uint32_t nonce;
    bool one_stream;  // the forward ran on the caller's stream only; its backward does too
};
constexpr int kSavedSlots = 64;
std::mutex g_saved_mu;
Saved g_saved[kSavedSlots];
int g_saved_next = 0;
uint32_t g_nonce = 0;

// Registers a saved forward and returns the nonce it leaves in the workspace.
// The nonce of a forward about to be enqueued (never 0).
uint32_t reserve_nonce() {
    std::lock_guard<std::mutex> lk(g_saved_mu);
    if (++g_nonce == 0) g_nonce = 1;  // 0: no saved forward
    return g_nonce;
}

// After the forward with `nonce` has been enqueued whole.
void remember_saved(const void* ws, uint64_t sig, bool one_stream, uint32_t nonce) {
    std::lock_guard<std::mutex> lk(g_saved_mu);
    for (int i = 0; i < kSavedSlots; ++i)
        if (g_saved[i].ws == ws) {
            g_saved[i].sig = sig;
            g_saved[i].nonce = nonce;
            g_saved[i].one_stream = one_stream;
            return;
        }
    g_saved[g_saved_next] = Saved{ws, sig, nonce, one_stream};
    g_saved_next = (g_saved_next + 1) % kSavedSlots;
}

void forget_saved(const void* ws) {
    std::lock_guard<std::mutex> lk(g_saved_mu);
    for (int i = 0; i < kSavedSlots; ++i)
        if (g_saved[i].ws == ws) g_saved[i].ws = nullptr;
}

bool was_saved(const void* ws, uint64_t sig, uint32_t* nonce, bool* one_stream) {
    std::lock_guard<std::mutex> lk(g_saved_mu);
    for (int i = 0; i < kSavedSlots; ++i)
        if (g_saved[i].ws == ws && ws != nullptr) {
            *nonce = g_saved[i].nonce;
            *one_stream = g_saved[i].one_stream;
            return g_saved[i].sig == sig;
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
    bool beside[kRing] = {};  // the slot's lo prep and raster ran beside the BVH build
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
// When the lo prep and raster ran beside the build, stage 2 spans from the
// start of the bake to the end of all three.
int32_t slot_times(int r, float* ms) {
    HIP_OR_FAIL(hipEventSynchronize(g_tim.ev[r][kStages - 1]));
    for (int k = 0; k < kStages; ++k) {
        float v = 0.f;
        if (k == 2 && g_tim.beside[r]) {
            HIP_OR_FAIL(hipEventElapsedTime(&v, g_tim.ev[r][0], g_tim.ev[r][3]));
        } else if (k < kStages - 1) {
            HIP_OR_FAIL(hipEventElapsedTime(&v, g_tim.ev[r][k], g_tim.ev[r][k + 1]));
        } else {
            HIP_OR_FAIL(hipEventElapsedTime(&v, g_tim.ev[r][0], g_tim.ev[r][kStages - 1]));
        }
        ms[k] = v;
    }
    return BAKE_OK;
}

int32_t check_workspace(const void* ws, size_t bytes, const Layout& L) {
    if (!ws) return fail(BAKE_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(BAKE_E_WORKSPACE, "workspace not 256-byte aligned");
    if (bytes < L.total)
        return fail(BAKE_E_WORKSPACE, "workspace has %zu bytes, needs %zu", bytes, L.total);
    return BAKE_OK;
}

// ---- the second stream --------------------------------------------------
// The low-poly prep and the UV raster do not depend on the BVH build (they
// share no workspace region with it), so the forward runs them on a second
// stream of the device, forked from and joined back to the caller's stream
// with events; under graph capture the fork and join become graph edges.  The
// stream and its events are created on the first forward of the device that
// is not being captured (a captured forward before that runs everything on
// the caller's stream).  Default priority.  The fork-join enqueue is
// serialised so that concurrent callers never see each other's event records.
constexpr int kMaxDevices = 64;
constexpr int64_t kSideMinFaces = 1 << 16;  // high-poly faces of a batch below which one stream is used
struct Side {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
Side g_side[kMaxDevices];
std::mutex g_side_mu;

Side* side_stream(hipStream_t s) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    Side& d = g_side[dev];
    if (d.s) return &d;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone) return nullptr;
    hipStream_t t = nullptr;
    hipEvent_t f = nullptr, j = nullptr;
    if (hipStreamCreateWithFlags(&t, hipStreamNonBlocking) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&f, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&j, hipEventDisableTiming) != hipSuccess) {
        if (f) (void)hipEventDestroy(f);
        (void)hipStreamDestroy(t);
        return nullptr;
    }
    d.fork = f;
    d.join = j;
    d.s = t;
    return &d;
}

// The forward launch sequence of a planned batch.
int32_t run_forward(Plan& P, const Opts& o, void* workspace, hipStream_t s) {
    char* ws = (char*)workspace;
    BatchHost H = host_view(P, ws);
    const Layout& L = P.L;
    const bool tim = (o.flags & BAKE_FLAG_TIMING) != 0;
    HIP_OR_FAIL(tim_record(tim, 0, s));
    // asset table + grid tables (one blob), then status, counters and batch
    // counters (contiguous from offset 0) to zero
    std::vector<char> blob(L.grads - L.table, 0);
    memcpy(blob.data(), P.A.data(), sizeof(AssetDev) * (size_t)L.n);
    memcpy(blob.data() + (L.gpf - L.table), P.gpf.data(), 4 * P.gpf.size());
    // the table, and the status, counters and BVH sort rows before it zeroed;
    // with BAKE_FLAG_SAVE the seal takes this forward's nonce in the same
    // launch (the backward checks it on the device: any later forward on the
    // workspace overwrites it, and the stream orders it before the backward)
    const bool save = (o.flags & BAKE_FLAG_SAVE) != 0;
    const uint32_t nonce = save ? reserve_nonce() : 0u;
    HIP_OR_FAIL(write_table(ws + L.table, blob.data(), (L.gpf - L.table) + 4 * P.gpf.size(), s, (uint32_t*)ws,
                            (int64_t)(L.table / 4), save ? (int64_t)(L.gcnt / 4 + kGcSeal) : -1, nonce));
    // small bakes run on one stream: there the fork and join cost more than
    // the overlap saves
    const bool one_stream = (o.flags & BAKE_FLAG_ONE_STREAM) != 0;
    std::unique_lock<std::mutex> side_lock(g_side_mu);
    Side* side = L.t_hf >= kSideMinFaces && !one_stream ? side_stream(s) : nullptr;
    if (side) {
        // the build, the longer chain, is enqueued first: kernels are handed
        // to the device one by one in the order they were enqueued (also on
        // a graph replay), so the chain enqueued second starts late
        HIP_OR_FAIL(hipEventRecord(side->fork, s));
        HIP_OR_FAIL(launch_bvh_build(H, s));
        HIP_OR_FAIL(hipStreamWaitEvent(side->s, side->fork, 0));
        HIP_OR_FAIL(launch_lo_prep(H, side->s));
        HIP_OR_FAIL(tim_record(tim, 1, side->s));
        HIP_OR_FAIL(launch_raster(H, side->s));
        HIP_OR_FAIL(tim_record(tim, 2, side->s));
        HIP_OR_FAIL(hipEventRecord(side->join, side->s));
        HIP_OR_FAIL(hipStreamWaitEvent(s, side->join, 0));
    } else {
        side_lock.unlock();
        HIP_OR_FAIL(launch_lo_prep(H, s));
        HIP_OR_FAIL(tim_record(tim, 1, s));
        HIP_OR_FAIL(launch_raster(H, s));
        HIP_OR_FAIL(tim_record(tim, 2, s));
        HIP_OR_FAIL(launch_bvh_build(H, s));
    }
    if (side_lock.owns_lock()) side_lock.unlock();
    if (tim) g_tim.beside[g_tim.next] = side != nullptr;
    HIP_OR_FAIL(tim_record(tim, 3, s));
    TravConfig tc = o.trav;
    tc.count = (o.flags & BAKE_FLAG_COUNT) != 0;
    tc.xcd = (o.flags & BAKE_FLAG_ONE_QUEUE) == 0;
    HIP_OR_FAIL(launch_traverse(H, tc, s));
    HIP_OR_FAIL(tim_record(tim, 4, s));
    HIP_OR_FAIL(launch_dilate(H, o.dilate, s));
    bool any_rgb8 = false;
    for (int a = 0; a < L.n; ++a) any_rgb8 = any_rgb8 || P.A[a].out_rgb8 != nullptr;
    if (any_rgb8) HIP_OR_FAIL(launch_rgb8(H, s));
    if (save) remember_saved(workspace, P.sig, one_stream, nonce);
    else forget_saved(workspace);
    HIP_OR_FAIL(tim_record(tim, 5, s));
    tim_commit(tim);
    return BAKE_OK;
}

int32_t run_backward(Plan& P, void* workspace, uint32_t nonce, bool one_stream, hipStream_t s) {
    char* ws = (char*)workspace;
    BatchHost H = host_view(P, ws);
    H.dev.seal = nonce;
    bool any_lo = false, any_hi = false;
    for (int a = 0; a < P.L.n; ++a) {
        any_lo = any_lo || P.G[a].grad_lo_V != nullptr;
        any_hi = any_hi || P.G[a].grad_hi_N != nullptr;
    }
    if (!any_lo && !any_hi) return BAKE_OK;
    // the gradient table, and the backward sort's super-tile rows zeroed
    HIP_OR_FAIL(write_table(ws + P.L.grads, P.G.data(), sizeof(AssetGrad) * (size_t)P.L.n, s,
                            (uint32_t*)(ws + P.L.bwd_sup), bwd_sort_zero_words(P.L)));
    std::lock_guard<std::mutex> side_lock(g_side_mu);
    Side* side = P.L.t_hf >= kSideMinFaces && !one_stream ? side_stream(s) : nullptr;
    if (side) {
        HIP_OR_FAIL(launch_backward(H, any_lo, any_hi, s, side->s, side->fork, side->join));
    } else {
        HIP_OR_FAIL(launch_backward(H, any_lo, any_hi, s));
    }
    return BAKE_OK;
}

bake_asset single_asset(const float* hi_V, int64_t n_hi_v, const int32_t* hi_F, int64_t n_hi_f,
                        const float* hi_N, const float* lo_V, int64_t n_lo_v, const int32_t* lo_F,
                        int64_t n_lo_f, const float* lo_UV, int32_t res, float max_dist) {
    bake_asset a;
    memset(&a, 0, sizeof a);
    a.hi_V = hi_V;
    a.n_hi_v = n_hi_v;
    a.hi_F = hi_F;
    a.n_hi_f = n_hi_f;
    a.hi_N = hi_N;
    a.lo_V = lo_V;
    a.n_lo_v = n_lo_v;
    a.lo_F = lo_F;
    a.n_lo_f = n_lo_f;
    a.lo_UV = lo_UV;
    a.res = res;
    a.max_dist = max_dist;
    return a;
}

int32_t read_counter_at(const void* workspace, int32_t asset, int32_t which, void* stream, int64_t* value_out) {
    if (!workspace || !value_out) return fail(BAKE_E_INVALID_ARG, "NULL argument");
    if (which < 0 || which > 3) return fail(BAKE_E_INVALID_ARG, "unknown counter %d", which);
    if (asset < 0 || asset >= kMaxAssets) return fail(BAKE_E_INVALID_ARG, "asset %d out of range", asset);
    hipStream_t s = (hipStream_t)stream;
    uint32_t v[kCntSlots];
    // per-asset counters start right after the 256-byte status block
    HIP_OR_FAIL(hipMemcpyAsync(v, (const char*)workspace + 256 + 4 * (size_t)kCntSlots * asset, sizeof v,
                               hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    if (which == 0) *value_out = v[kCntRays];
    else if (which == 1) *value_out = (int64_t)v[kCntBoxLo] | ((int64_t)v[kCntBoxLo + 1] << 32);
    else if (which == 2) *value_out = (int64_t)v[kCntTriLo] | ((int64_t)v[kCntTriLo + 1] << 32);
    else *value_out = (int64_t)v[kCntIterLo] | ((int64_t)v[kCntIterLo + 1] << 32);
    return BAKE_OK;
}

// ---- the scratch array of bake_normals_noalloc ------------------------------
// For callers that cannot allocate device memory, the bake's workspace is a
// fixed array in the library's own device memory, one per GPU (the runtime
// places it with the code object; it lives until the process ends).  Host
// code must never use the array's name as a device address: the device
// address is resolved once per device with hipGetSymbolAddress, with that
// device current, on the entry point's first call there, and every launch and
// fill takes that address.  Calls on one GPU share the array: the bake
// clears what must start at zero (its status block and counters) at the start
// of every call, and calls that overlap on one GPU race.
constexpr size_t kNoAllocBytes = (size_t)BAKE_NOALLOC_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

int32_t noalloc_scratch(void** out) {
    int dev = -1;
    HIP_OR_FAIL(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(BAKE_E_UNSUPPORTED, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_OR_FAIL(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255) != 0) return fail(BAKE_E_HIP, "scratch array address %p unusable", p);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BAKE_OK;
}

// ---- hidden-face removal (Sec. 6.2) ----------------------------------------
// The workspace of a visibility pass: the batch-of-one plan whose asset has
// the mesh as its high-poly and no low-poly (its BVH build is the bake's),
// then the flood fill's arrays and the camera rays' spill columns.
struct VisLayout {
    size_t deg, off, cur, adj, vis, ext, front0, front1, scan_tmp, spill, total;
};

int32_t plan_visibility(int64_t nv, int64_t nf, Plan* P, VisLayout* V) {
    Sizes z;
    z.nhv = nv;
    z.nhf = nf;
    z.nlv = 0;
    z.nlf = 0;
    z.res = 1;
    int32_t rc = make_plan(&z, 1, 0, P);
    if (rc) return rc;
    size_t off = align256(P->L.total);
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    V->deg = take(4 * (size_t)(nv + 1));
    V->off = take(4 * (size_t)(nv + 1));
    V->cur = take(4 * (size_t)(nv + 1));
    V->adj = take(4 * (size_t)(3 * nf + 1));
    V->vis = take(4 * (size_t)(nf + 1));
    V->ext = take(4 * (size_t)(nf + 1));
    V->front0 = take(4 * (size_t)(nf + 1));
    V->front1 = take(4 * (size_t)(nf + 1));
    V->scan_tmp = take(4 * (size_t)(scan_tmp_elems(nv + 1) + 1));
    V->spill = take(4 * (size_t)kMaxDepth * (size_t)kMaxLanes);
    V->total = off;
    return BAKE_OK;
}

// ---- backprojection precompute (Sec. 7.4, TextureGen Postprocessing) ----
// A batch of one asset whose low-poly and high-poly are both the textured
// mesh (its atlas rasterised as in the bake, its BVH for the depth rays),
// then the views' depth buffers and the depth rays' spill columns.
struct MapLayout {
    size_t depth, spill, total;
};

int32_t plan_view_maps(int64_t nv, int64_t nf, int32_t res, int32_t n_views, int32_t img_res, Plan* P,
                       MapLayout* M) {
    Sizes z;
    z.nhv = z.nlv = nv;
    z.nhf = z.nlf = nf;
    z.res = res;
    int32_t rc = make_plan(&z, 1, 0, P);
    if (rc) return rc;
    if (n_views < 1 || n_views > 4096) return fail(BAKE_E_INVALID_ARG, "n_views %d outside [1, 4096]", n_views);
    if (img_res < 1 || img_res > 16384) return fail(BAKE_E_INVALID_ARG, "img_res %d outside [1, 16384]", img_res);
    size_t off = align256(P->L.total);
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    M->depth = take(4 * (size_t)n_views * (size_t)img_res * (size_t)img_res);
    M->spill = take(4 * (size_t)kMaxDepth * (size_t)kMaxLanes);
    M->total = off;
    return BAKE_OK;
}

}  // namespace

extern "C" {

void bake_default_options(bake_options* opt) {
    if (!opt) return;
    memset(opt, 0, sizeof *opt);
    opt->dilate_passes = 2;
    opt->trav_mode = -1;
}

const char* bake_last_error(void) { return g_err; }

const char* bake_version(void) { return "paper_2605_26137_amd bake 0.2 (gfx950)"; }

int32_t bake_workspace_size(int64_t n_hi_v, int64_t n_hi_f, int64_t n_lo_v, int64_t n_lo_f,
                            int32_t res, const bake_options* opt, size_t* bytes_out) {
    g_err[0] = 0;
    if (!bytes_out) return fail(BAKE_E_INVALID_ARG, "bytes_out is NULL");
    Opts o;
    int32_t rc = parse_opts(opt, &o);
    if (rc) return rc;
    Sizes z{n_hi_v, n_hi_f, n_lo_v, n_lo_f, res};
    Plan P;
    if ((rc = make_plan(&z, 1, o.flags, &P))) return rc;
    *bytes_out = P.L.total;
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
    Sizes z{n_hi_v, n_hi_f, n_lo_v, n_lo_f, res};
    Plan P;
    if ((rc = make_plan(&z, 1, o.flags, &P))) return rc;
    const Layout& L = P.L;
    const size_t tex = (size_t)res * res;
    switch (which) {
        case BAKE_VIEW_RAYS: *offset_out = L.rays; *bytes_out = 16 * tex; break;
        case BAKE_VIEW_HITS:
            if (!(o.flags & BAKE_FLAG_SAVE)) return fail(BAKE_E_INVALID_ARG, "hits need BAKE_FLAG_SAVE");
            *offset_out = L.hits; *bytes_out = 16 * tex; break;
        case BAKE_VIEW_FACEMAP: *offset_out = L.facemap; *bytes_out = 4 * tex; break;
        case BAKE_VIEW_LO_N: *offset_out = L.lo_n; *bytes_out = 16 * (size_t)n_lo_v; break;
        case BAKE_VIEW_SORTED: *offset_out = L.keys0; *bytes_out = 4 * (size_t)n_hi_f; break;
        case BAKE_VIEW_SORTED_IDX: *offset_out = L.vals0; *bytes_out = 4 * (size_t)n_hi_f; break;
        case BAKE_VIEW_NODES:
            *offset_out = L.nodes_c; *bytes_out = 32 * (size_t)std::max<int64_t>(n_hi_f - 1, 0); break;
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
    bake_asset a = single_asset(hi_V, n_hi_v, hi_F, n_hi_f, hi_N, lo_V, n_lo_v, lo_F, n_lo_f, lo_UV, res,
                                max_dist);
    a.out_map = out_map;
    a.out_hit = out_hit;
    a.out_rgb8 = o.rgb8;
    Plan P;
    if ((rc = plan_batch(&a, 1, o.flags, &P))) return rc;
    if ((rc = validate_asset(a, 0))) return rc;
    if (!out_map || !out_hit) return fail(BAKE_E_INVALID_ARG, "out_map / out_hit is NULL");
    if ((rc = check_workspace(workspace, workspace_bytes, P.L))) return rc;
    fill_pointers(&a, &P);
    return run_forward(P, o, workspace, (hipStream_t)stream);
}

int32_t bake_normals_noalloc(const float* hi_V, int64_t n_hi_v, const int32_t* hi_F, int64_t n_hi_f,
                             const float* hi_N, const float* lo_V, int64_t n_lo_v, const int32_t* lo_F,
                             int64_t n_lo_f, const float* lo_UV, int32_t res, float max_dist, float* out_map,
                             int32_t* out_hit, const bake_options* opt, void* stream) {
    g_err[0] = 0;
    Opts o;
    int32_t rc = parse_opts(opt, &o);
    if (rc) return rc;
    if (o.flags & (BAKE_FLAG_SAVE | BAKE_FLAG_TIMING | BAKE_FLAG_COUNT))
        return fail(BAKE_E_INVALID_ARG,
                    "bake_normals_noalloc takes no BAKE_FLAG_SAVE, BAKE_FLAG_TIMING or BAKE_FLAG_COUNT");
    o.flags |= BAKE_FLAG_ONE_STREAM;  // the second stream and its events would be created on first use
    bake_asset a = single_asset(hi_V, n_hi_v, hi_F, n_hi_f, hi_N, lo_V, n_lo_v, lo_F, n_lo_f, lo_UV, res,
                                max_dist);
    a.out_map = out_map;
    a.out_hit = out_hit;
    a.out_rgb8 = o.rgb8;
    Plan P;
    if ((rc = plan_batch(&a, 1, o.flags, &P))) return rc;
    if ((rc = validate_asset(a, 0))) return rc;
    if (!out_map || !out_hit) return fail(BAKE_E_INVALID_ARG, "out_map / out_hit is NULL");
    if (P.L.total > kNoAllocBytes)
        return fail(BAKE_E_WORKSPACE,
                    "this bake needs %zu bytes of scratch; bake_normals_noalloc holds %zu (BAKE_NOALLOC_BYTES): "
                    "use bake_normals with a workspace",
                    P.L.total, kNoAllocBytes);
    void* ws = nullptr;
    if ((rc = noalloc_scratch(&ws))) return rc;
    fill_pointers(&a, &P);
    return run_forward(P, o, ws, (hipStream_t)stream);
}

int32_t bake_normals_backward(const float* hi_V, int64_t n_hi_v, const int32_t* hi_F,
                              int64_t n_hi_f, const float* hi_N, const float* lo_V, int64_t n_lo_v,
                              const int32_t* lo_F, int64_t n_lo_f, const float* lo_UV, int32_t res,
                              float max_dist, const float* grad_map, float* grad_lo_V,
                              float* grad_hi_N, void* workspace, size_t workspace_bytes,
                              void* stream) {
    g_err[0] = 0;
    bake_asset a = single_asset(hi_V, n_hi_v, hi_F, n_hi_f, hi_N, lo_V, n_lo_v, lo_F, n_lo_f, lo_UV, res,
                                max_dist);
    a.grad_map = grad_map;
    a.grad_lo_V = grad_lo_V;
    a.grad_hi_N = grad_hi_N;
    return bake_normals_batched_backward(&a, 1, workspace, workspace_bytes, stream);
}

int32_t bake_batch_workspace_size(const bake_asset* assets, int32_t n_assets, const bake_options* opt,
                                  size_t* bytes_out) {
    g_err[0] = 0;
    if (!bytes_out) return fail(BAKE_E_INVALID_ARG, "bytes_out is NULL");
    Opts o;
    int32_t rc = parse_opts(opt, &o);
    if (rc) return rc;
    Plan P;
    if ((rc = plan_batch(assets, n_assets, o.flags, &P))) return rc;
    *bytes_out = P.L.total;
    return BAKE_OK;
}

int32_t bake_normals_batched(const bake_asset* assets, int32_t n_assets, const bake_options* opt,
                             void* workspace, size_t workspace_bytes, void* stream) {
    g_err[0] = 0;
    Opts o;
    int32_t rc = parse_opts(opt, &o);
    if (rc) return rc;
    if (o.rgb8) return fail(BAKE_E_INVALID_ARG, "batches take RGB8 outputs per asset (opt->out_rgb8 must be NULL)");
    Plan P;
    if ((rc = plan_batch(assets, n_assets, o.flags, &P))) return rc;
    for (int a = 0; a < n_assets; ++a) {
        if ((rc = validate_asset(assets[a], a))) return rc;
        if (!assets[a].out_map || !assets[a].out_hit)
            return fail(BAKE_E_INVALID_ARG, "asset %d: out_map / out_hit is NULL", a);
    }
    if ((rc = check_workspace(workspace, workspace_bytes, P.L))) return rc;
    fill_pointers(assets, &P);
    return run_forward(P, o, workspace, (hipStream_t)stream);
}

int32_t bake_normals_batched_backward(const bake_asset* assets, int32_t n_assets, void* workspace,
                                      size_t workspace_bytes, void* stream) {
    g_err[0] = 0;
    Plan P;
    int32_t rc = plan_batch(assets, n_assets, BAKE_FLAG_SAVE, &P);
    if (rc) return rc;
    for (int a = 0; a < n_assets; ++a) {
        if ((rc = validate_asset(assets[a], a))) return rc;
        if (!assets[a].grad_map && (assets[a].grad_lo_V || assets[a].grad_hi_N))
            return fail(BAKE_E_INVALID_ARG, "asset %d: grad_map is NULL", a);
    }
    if ((rc = check_workspace(workspace, workspace_bytes, P.L))) return rc;
    uint32_t nonce = 0;
    bool one_stream = false;
    if (!was_saved(workspace, P.sig, &nonce, &one_stream))
        return fail(BAKE_E_STATE, "no forward bake with BAKE_FLAG_SAVE and these sizes used this workspace");
    fill_pointers(assets, &P);
    return run_backward(P, workspace, nonce, one_stream, (hipStream_t)stream);
}

int32_t bake_autotune(const bake_asset* assets, int32_t n_assets, const bake_options* base, int32_t reps,
                      void* workspace, size_t workspace_bytes, void* stream, bake_options* best_out,
                      float* ms_out) {
    g_err[0] = 0;
    if (!best_out) return fail(BAKE_E_INVALID_ARG, "best_out is NULL");
    if (reps < 1 || reps > 64) return fail(BAKE_E_INVALID_ARG, "reps %d outside [1, 64]", reps);
    bake_options opt;
    if (base) opt = *base;
    else bake_default_options(&opt);
    static const int blocks[3] = {64, 128, 256}, stacks[3] = {8, 16, 32};
    float best = INFINITY;
    bake_options best_opt = opt;
    int idx = 0;
    for (int bi = 0; bi < 3; ++bi)
        for (int si = 0; si < 3; ++si)
            for (int pe = 0; pe < 4; ++pe, ++idx) {
                bake_options o = opt;
                o.trav_block = blocks[bi];
                o.trav_stack = stacks[si];
                o.trav_mode = pe;
                o.flags = (opt.flags & ~(uint32_t)BAKE_FLAG_COUNT) | BAKE_FLAG_TIMING;
                std::vector<float> t(reps);
                for (int r = 0; r < reps; ++r) {
                    int32_t rc = bake_normals_batched(assets, n_assets, &o, workspace, workspace_bytes, stream);
                    if (rc) return rc;
                    float ms[kStages];
                    if ((rc = slot_times((g_tim.next + kRing - 1) % kRing, ms))) return rc;
                    t[r] = ms[3];
                }
                std::sort(t.begin(), t.end());
                const float med = t[reps / 2];
                if (ms_out) ms_out[idx] = med;
                if (med < best) {
                    best = med;
                    best_opt = opt;
                    best_opt.trav_block = blocks[bi];
                    best_opt.trav_stack = stacks[si];
                    best_opt.trav_mode = pe;
                }
            }
    *best_out = best_opt;
    return BAKE_OK;
}

int32_t bake_visibility_workspace_size(int64_t n_v, int64_t n_f, size_t* bytes_out) {
    g_err[0] = 0;
    if (!bytes_out) return fail(BAKE_E_INVALID_ARG, "bytes_out is NULL");
    Plan P;
    VisLayout VL;
    int32_t rc = plan_visibility(n_v, n_f, &P, &VL);
    if (rc) return rc;
    *bytes_out = VL.total;
    return BAKE_OK;
}

int32_t bake_visibility(const float* V, const int32_t* F, int64_t n_v, int64_t n_f, const float* eyes,
                        int32_t n_views, const float* target, float tan_half_fov, int32_t res, float t_far,
                        uint32_t flags, uint8_t* visible_out, uint8_t* exterior_out, int32_t* first_hit_out,
                        void* workspace, size_t workspace_bytes, void* stream) {
    g_err[0] = 0;
    if (n_v > 0 && !V) return fail(BAKE_E_INVALID_ARG, "V is NULL");
    if (n_f > 0 && (!F || !visible_out)) return fail(BAKE_E_INVALID_ARG, "F / visible_out is NULL");
    if (n_views < 1 || n_views > (1 << 20)) return fail(BAKE_E_INVALID_ARG, "n_views %d outside [1, 2^20]", n_views);
    if (!eyes || !target) return fail(BAKE_E_INVALID_ARG, "eyes / target is NULL");
    if (res < 1 || res > 16384) return fail(BAKE_E_INVALID_ARG, "res %d outside [1, 16384]", res);
    if (!(tan_half_fov > 0.f) || !(tan_half_fov < INFINITY))
        return fail(BAKE_E_INVALID_ARG, "tan_half_fov must be finite and > 0");
    if (!(t_far > 0.f) || !(t_far < INFINITY)) return fail(BAKE_E_INVALID_ARG, "t_far must be finite and > 0");
    for (int k = 0; k < 3; ++k)
        if (!(fabsf(target[k]) < INFINITY)) return fail(BAKE_E_INVALID_ARG, "target must be finite");
    if ((flags & ~(uint32_t)(BAKE_FLAG_COUNT | BAKE_FLAG_TIMING)) != 0)
        return fail(BAKE_E_INVALID_ARG, "flags 0x%x: only BAKE_FLAG_COUNT and BAKE_FLAG_TIMING apply", flags);
    Plan P;
    VisLayout VL;
    int32_t rc = plan_visibility(n_v, n_f, &P, &VL);
    if (rc) return rc;
    if (!workspace) return fail(BAKE_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(BAKE_E_WORKSPACE, "workspace not 256-byte aligned");
    if (workspace_bytes < VL.total)
        return fail(BAKE_E_WORKSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, VL.total);
    AssetDev& d = P.A[0];
    d.hi_V = V;
    d.hi_F = F;
    d.max_dist = t_far;
    P.G.assign(1, AssetGrad{});
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)workspace;
    BatchHost H = host_view(P, ws);
    const Layout& L = P.L;
    const bool tim = (flags & BAKE_FLAG_TIMING) != 0;
    HIP_OR_FAIL(tim_record(tim, 0, s));
    std::vector<char> blob(L.grads - L.table, 0);
    memcpy(blob.data(), P.A.data(), sizeof(AssetDev));
    memcpy(blob.data() + (L.gpf - L.table), P.gpf.data(), 4 * P.gpf.size());
    // the table, and the status, counters and BVH sort rows before it zeroed
    HIP_OR_FAIL(write_table(ws + L.table, blob.data(), (L.gpf - L.table) + 4 * P.gpf.size(), s, (uint32_t*)ws,
                            (int64_t)(L.table / 4)));
    forget_saved(workspace);
    HIP_OR_FAIL(tim_record(tim, 1, s));
    HIP_OR_FAIL(launch_bvh_build(H, s));
    HIP_OR_FAIL(tim_record(tim, 2, s));
    uint32_t* vis = (uint32_t*)(ws + VL.vis);
    HIP_OR_FAIL(fill_u32(vis, 0, n_f, s));
    VisRun vr{};
    vr.eyes = eyes;
    for (int k = 0; k < 3; ++k) vr.target[k] = target[k];
    vr.tan_half = tan_half_fov;
    vr.n_views = n_views;
    vr.res = res;
    vr.visible = vis;
    vr.first_hit = first_hit_out;
    vr.depth = nullptr;
    vr.spill = (int32_t*)(ws + VL.spill);
    vr.spill_lanes = kMaxLanes;
    vr.count = (flags & BAKE_FLAG_COUNT) != 0;
    HIP_OR_FAIL(launch_visibility_rays(H, vr, s));
    HIP_OR_FAIL(tim_record(tim, 3, s));
    FillRun fr;
    fr.deg = (uint32_t*)(ws + VL.deg);
    fr.off = (uint32_t*)(ws + VL.off);
    fr.cur = (uint32_t*)(ws + VL.cur);
    fr.adj = (uint32_t*)(ws + VL.adj);
    fr.ext = (uint32_t*)(ws + VL.ext);
    fr.front0 = (uint32_t*)(ws + VL.front0);
    fr.front1 = (uint32_t*)(ws + VL.front1);
    fr.scan_tmp = (uint32_t*)(ws + VL.scan_tmp);
    fr.visible = vis;
    fr.visible_out = visible_out;
    fr.exterior_out = exterior_out;
    if (n_f > 0) HIP_OR_FAIL(launch_flood_fill(H, fr, s));
    HIP_OR_FAIL(tim_record(tim, 4, s));
    HIP_OR_FAIL(tim_record(tim, 5, s));
    tim_commit(tim);
    return BAKE_OK;
}

int32_t bake_view_maps_workspace_size(int64_t n_v, int64_t n_f, int32_t res, int32_t n_views, int32_t img_res,
                                      size_t* bytes_out) {
    g_err[0] = 0;
    if (!bytes_out) return fail(BAKE_E_INVALID_ARG, "bytes_out is NULL");
    Plan P;
    MapLayout M;
    int32_t rc = plan_view_maps(n_v, n_f, res, n_views, img_res, &P, &M);
    if (rc) return rc;
    *bytes_out = M.total;
    return BAKE_OK;
}

int32_t bake_view_maps(const float* V, const int32_t* F, const float* UV, int64_t n_v, int64_t n_f, int32_t res,
                       const float* eyes, int32_t n_views, const float* target, float tan_half_fov,
                       int32_t img_res, float t_far, float depth_tol, uint32_t flags, float* uv_out,
                       float* inc_out, float* depth_out, void* workspace, size_t workspace_bytes, void* stream) {
    g_err[0] = 0;
    if (n_v > 0 && !V) return fail(BAKE_E_INVALID_ARG, "V is NULL");
    if (n_f > 0 && (!F || !UV)) return fail(BAKE_E_INVALID_ARG, "F / UV is NULL");
    if (!eyes || !target || !uv_out || !inc_out) return fail(BAKE_E_INVALID_ARG, "eyes / target / outputs NULL");
    if (!(tan_half_fov > 0.f) || !(tan_half_fov < INFINITY))
        return fail(BAKE_E_INVALID_ARG, "tan_half_fov must be finite and > 0");
    if (!(t_far > 0.f) || !(t_far < INFINITY)) return fail(BAKE_E_INVALID_ARG, "t_far must be finite and > 0");
    if (!(depth_tol >= 0.f) || !(depth_tol < INFINITY))
        return fail(BAKE_E_INVALID_ARG, "depth_tol must be finite and >= 0");
    for (int k = 0; k < 3; ++k)
        if (!(fabsf(target[k]) < INFINITY)) return fail(BAKE_E_INVALID_ARG, "target must be finite");
    if ((flags & ~(uint32_t)(BAKE_FLAG_COUNT | BAKE_FLAG_TIMING)) != 0)
        return fail(BAKE_E_INVALID_ARG, "flags 0x%x: only BAKE_FLAG_COUNT and BAKE_FLAG_TIMING apply", flags);
    Plan P;
    MapLayout M;
    int32_t rc = plan_view_maps(n_v, n_f, res, n_views, img_res, &P, &M);
    if (rc) return rc;
    if (!workspace) return fail(BAKE_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(BAKE_E_WORKSPACE, "workspace not 256-byte aligned");
    if (workspace_bytes < M.total)
        return fail(BAKE_E_WORKSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, M.total);
    AssetDev& d = P.A[0];
    d.hi_V = d.lo_V = V;
    d.hi_F = d.lo_F = F;
    d.lo_UV = UV;
    d.max_dist = t_far;
    P.G.assign(1, AssetGrad{});
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)workspace;
    BatchHost H = host_view(P, ws);
    const Layout& L = P.L;
    const bool tim = (flags & BAKE_FLAG_TIMING) != 0;
    HIP_OR_FAIL(tim_record(tim, 0, s));
    std::vector<char> blob(L.grads - L.table, 0);
    memcpy(blob.data(), P.A.data(), sizeof(AssetDev));
    memcpy(blob.data() + (L.gpf - L.table), P.gpf.data(), 4 * P.gpf.size());
    // the table, and the status, counters and BVH sort rows before it zeroed
    HIP_OR_FAIL(write_table(ws + L.table, blob.data(), (L.gpf - L.table) + 4 * P.gpf.size(), s, (uint32_t*)ws,
                            (int64_t)(L.table / 4)));
    forget_saved(workspace);
    HIP_OR_FAIL(launch_lo_prep(H, s));
    HIP_OR_FAIL(launch_raster(H, s));
    HIP_OR_FAIL(tim_record(tim, 1, s));
    HIP_OR_FAIL(launch_bvh_build(H, s));
    HIP_OR_FAIL(tim_record(tim, 2, s));
    float* depth = depth_out ? depth_out : (float*)(ws + M.depth);
    VisRun vr{};
    vr.eyes = eyes;
    for (int k = 0; k < 3; ++k) vr.target[k] = target[k];
    vr.tan_half = tan_half_fov;
    vr.n_views = n_views;
    vr.res = img_res;
    vr.visible = nullptr;
    vr.first_hit = nullptr;
    vr.depth = depth;
    vr.spill = (int32_t*)(ws + M.spill);
    vr.spill_lanes = kMaxLanes;
    vr.count = (flags & BAKE_FLAG_COUNT) != 0;
    HIP_OR_FAIL(launch_visibility_rays(H, vr, s));
    HIP_OR_FAIL(tim_record(tim, 3, s));
    const int64_t tex = (int64_t)res * res;
    HIP_OR_FAIL(fill_u32((uint32_t*)uv_out, 0xBF800000u, 2 * (int64_t)n_views * tex, s));  // -1.0f
    HIP_OR_FAIL(fill_u32((uint32_t*)inc_out, 0u, (int64_t)n_views * tex, s));
    MapRun mr{};
    mr.eyes = eyes;
    for (int k = 0; k < 3; ++k) mr.target[k] = target[k];
    mr.tan_half = tan_half_fov;
    mr.n_views = n_views;
    mr.img_res = img_res;
    mr.depth = depth;
    mr.tol = depth_tol;
    mr.uv_out = uv_out;
    mr.inc_out = inc_out;
    HIP_OR_FAIL(launch_view_maps(H, mr, s));
    HIP_OR_FAIL(tim_record(tim, 4, s));
    HIP_OR_FAIL(tim_record(tim, 5, s));
    tim_commit(tim);
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
    return read_counter_at(workspace, 0, which, stream, value_out);
}

int32_t bake_read_asset_counter(const void* workspace, int32_t asset, int32_t which, void* stream,
                                int64_t* value_out) {
    g_err[0] = 0;
    return read_counter_at(workspace, asset, which, stream, value_out);
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

// ---- mesh simplification (Sec. 6.1) ---------------------------------------

int32_t bake_qem_workspace_size(int64_t n_v, int64_t n_f, size_t* bytes_out) {
    g_err[0] = 0;
    if (!bytes_out) return fail(BAKE_E_INVALID_ARG, "bytes_out is NULL");
    if (n_v < 0 || n_f < 0) return fail(BAKE_E_INVALID_ARG, "negative count");
    if (n_v >= ((int64_t)1 << 28) || n_f >= ((int64_t)1 << 28))
        return fail(BAKE_E_UNSUPPORTED, "counts must be < 2^28");
    QemLayout L;
    *bytes_out = qem_layout(n_v, n_f, &L);
    return BAKE_OK;
}

static int32_t qem_common(const float* V, const int32_t* F, int64_t n_v, int64_t n_f, uint32_t flags,
                          void* workspace, size_t workspace_bytes, QemLayout* L) {
    if (n_v < 0 || n_f < 0) return fail(BAKE_E_INVALID_ARG, "negative count");
    if (n_v >= ((int64_t)1 << 28) || n_f >= ((int64_t)1 << 28))
        return fail(BAKE_E_UNSUPPORTED, "counts must be < 2^28");
    if (n_v > 0 && !V) return fail(BAKE_E_INVALID_ARG, "V is NULL");
    if (n_f > 0 && !F) return fail(BAKE_E_INVALID_ARG, "F is NULL");
    if ((flags & ~BAKE_QEM_MIDPOINT) != 0) return fail(BAKE_E_INVALID_ARG, "unknown flag bits 0x%x", flags);
    const size_t need = qem_layout(n_v, n_f, L);
    if (!workspace) return fail(BAKE_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(BAKE_E_WORKSPACE, "workspace not 256-byte aligned");
    if (workspace_bytes < need) return fail(BAKE_E_WORKSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    return BAKE_OK;
}

int32_t bake_qem_simplify(const float* V, const int32_t* F, int64_t n_v, int64_t n_f, int64_t target_faces,
                          double rho, int32_t max_rounds, uint32_t flags, float* V_out, int32_t* F_out,
                          int64_t* counts_out, int32_t* rounds_out, int64_t* stats_out, float* times_ms_out,
                          void* workspace, size_t workspace_bytes, void* stream) {
    g_err[0] = 0;
    if (target_faces < 4) return fail(BAKE_E_INVALID_ARG, "target_faces %lld < 4", (long long)target_faces);
    if (!(rho > 0.0 && rho <= 1.0)) return fail(BAKE_E_INVALID_ARG, "rho must lie in (0, 1]");
    if (max_rounds < 0) return fail(BAKE_E_INVALID_ARG, "max_rounds < 0");
    if (!counts_out || !rounds_out) return fail(BAKE_E_INVALID_ARG, "counts_out / rounds_out is NULL");
    if ((n_v > 0 && !V_out) || (n_f > 0 && !F_out)) return fail(BAKE_E_INVALID_ARG, "V_out / F_out is NULL");
    QemLayout L;
    int32_t rc = qem_common(V, F, n_v, n_f, flags, workspace, workspace_bytes, &L);
    if (rc) return rc;
    uint32_t status = 0;
    HIP_OR_FAIL(qem_simplify_run(L, (char*)workspace, V, F, target_faces, rho, max_rounds,
                                 (flags & BAKE_QEM_MIDPOINT) ? 1 : 0, V_out, F_out, counts_out, rounds_out, stats_out,
                                 times_ms_out, &status, (hipStream_t)stream));
    if (status) return fail(BAKE_E_INDEX, "a face has an index outside [0, n_v) or a repeated vertex");
    return BAKE_OK;
}

int32_t bake_qem_edges(const float* V, const int32_t* F, int64_t n_v, int64_t n_f, uint32_t flags, int64_t cap,
                       int32_t* edges_out, uint8_t* valid_out, int32_t* faces_out, double* cost_out, double* p_out,
                       double* Q_out, int64_t* n_edges_out, void* workspace, size_t workspace_bytes, void* stream) {
    g_err[0] = 0;
    if (!n_edges_out) return fail(BAKE_E_INVALID_ARG, "n_edges_out is NULL");
    if (cap < 0) return fail(BAKE_E_INVALID_ARG, "cap < 0");
    if (cap > 0 && (!edges_out || !valid_out || !faces_out || !cost_out || !p_out))
        return fail(BAKE_E_INVALID_ARG, "an edge output is NULL");
    QemLayout L;
    int32_t rc = qem_common(V, F, n_v, n_f, flags, workspace, workspace_bytes, &L);
    if (rc) return rc;
    uint32_t status = 0;
    HIP_OR_FAIL(qem_edges_run(L, (char*)workspace, V, F, (flags & BAKE_QEM_MIDPOINT) ? 1 : 0, Q_out, cap, edges_out,
                              valid_out, faces_out, cost_out, p_out, &status, n_edges_out, (hipStream_t)stream));
    if (status) return fail(BAKE_E_INDEX, "a face has an index outside [0, n_v) or a repeated vertex");
    if (*n_edges_out > cap)
        return fail(BAKE_E_INVALID_ARG, "the mesh has %lld edges, cap is %lld", (long long)*n_edges_out,
                    (long long)cap);
    return BAKE_OK;
}

}  // extern "C"
