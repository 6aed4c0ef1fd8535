/*
 * FP64 CPU oracle for tangent-space normal baking.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no source, header, table or helper with the GPU
 * library.
 *
 * What it computes follows the paper's bake (Sec. 6.4 "Normal Map Baking"):
 * rasterise the low-poly into its own UV space to get, per valid texel, a
 * world position, a smooth normal and a tangent frame; find the corresponding
 * point on the high-poly; interpolate the high-poly smooth normal there with the
 * hit's barycentric weights; reject far or unreliable correspondences with the
 * neutral normal (0,0,1); project the hit normal into the texel's tangent frame;
 * dilate at chart borders.  The correspondence query is a two-sided ray cast
 * along the interpolated low-poly normal, nearest |t| within +-max_dist, ties to
 * the lower triangle index; the paper's own form, the closest point of the
 * high-poly surface within a distance bound, is the second query below.
 *
 * The hidden-face removal of Sec. 6.2 (visibility rays from viewpoints around
 * the mesh and a normal-gated flood fill over shared edges) reuses the same
 * triangle test and BVH.
 *
 * Everything is plain: brute force over every texel and every triangle,
 * FP64 arithmetic, no blocking or reordering beyond what the definitions say.
 * A separate, equally plain FP64 BVH (median split) answers the same query and
 * is pinned against the brute force.
 *
 * Conventions (readings where the paper is silent):
 *   texel (i, j): centre u = (j + 1/2)/res, v = (i + 1/2)/res, row-major [i][j];
 *   coverage: corners snapped to 1/256 texel, X = rint(u*res*256); integer edge
 *     functions at the centre (256j+128, 256i+128); inside iff all >= 0 or all
 *     <= 0 and their sum != 0; the lowest face index wins an overlap;
 *   low-poly vertex normal: normalised sum of unnormalised incident face cross
 *     products (area weighted);
 *   tangent frame from the snapped UV deltas; per texel Gram-Schmidt against the
 *     interpolated normal; bitangent = h_f * (d x T');
 *   status: >= 0 hit id, -1 miss, -2 unreliable, -3 uncovered;
 *   hit rules (the `rule` argument of the ray queries):
 *     RULE_PLAIN, the plain definition of the nearest hit: a triangle is hit
 *       when the three signed volumes of the line against its edges share a
 *       sign (zeros allowed, not all zero); among hits with |t| <= max_dist the
 *       winner minimises (|t|, index);
 *     RULE_ROBUST, the convention the GPU library implements: a triangle is
 *       hit when the line crosses its plane at barycentric weights all >=
 *       -EDGE_EPS (a relative edge tolerance, so a line grazing a shared edge
 *       or vertex hits every face there); the winner minimises
 *       (floor(|t| / w), index) with the distance quantum w = max_dist * 2^-20,
 *       so hits whose distances agree to within the quantum resolve to the
 *       lower triangle index.  It differs from the plain rule only on lines
 *       passing within the tolerance of an edge and on distances within a
 *       quantum: the tests measure that difference on the workloads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_EINVAL -1

/* relative edge tolerance (in barycentric units) and distance quantum of the
 * robust rule */
#define EDGE_EPS (1.0 / 16384.0)
#define T_QUANT_BITS 20

#define RULE_PLAIN 0
#define RULE_ROBUST 1

#define ST_MISS -1
#define ST_UNREL -2
#define ST_UNCOV -3

typedef struct { double x, y, z; } v3;

static v3 mk(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 scl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 cross(v3 a, v3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static double norm(v3 a) { return sqrt(dot(a, a)); }
static v3 ld3f(const float *p, int64_t i) { return mk(p[3 * i], p[3 * i + 1], p[3 * i + 2]); }
static v3 ld3d(const double *p, int64_t i) { return mk(p[3 * i], p[3 * i + 1], p[3 * i + 2]); }
static void st3d(double *p, int64_t i, v3 a) { p[3 * i] = a.x; p[3 * i + 1] = a.y; p[3 * i + 2] = a.z; }

static int64_t floordiv(int64_t a, int64_t b) {  /* b > 0 */
    int64_t q = a / b;
    if ((a % b) != 0 && a < 0) q -= 1;
    return q;
}

int orc_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

/* ------------------------------------------------------------------------ */
/* Low-poly smooth normals (G-buffer "smooth normal", Sec. 6.4)              */
/* ------------------------------------------------------------------------ */

/* n_v = normalise(sum over faces containing v of (V1-V0) x (V2-V0)).
 * Writes the normalised normal and a validity flag (0 where the sum is 0). */
int orc_lo_normals(const float *V, int64_t nv, const int32_t *F, int64_t nf,
                   double *n_out, uint8_t *valid_out) {
    if (!V || !F || !n_out || nv < 0 || nf < 0) return ORC_EINVAL;
    double *acc = (double *)calloc((size_t)(3 * (nv > 0 ? nv : 1)), sizeof(double));
    for (int64_t f = 0; f < nf; ++f) {
        int32_t a = F[3 * f], b = F[3 * f + 1], c = F[3 * f + 2];
        if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv) { free(acc); return ORC_EINVAL; }
        v3 A = ld3f(V, a), B = ld3f(V, b), C = ld3f(V, c);
        v3 cr = cross(sub(B, A), sub(C, A));
        int32_t id[3] = {a, b, c};
        for (int k = 0; k < 3; ++k) st3d(acc, id[k], add(ld3d(acc, id[k]), cr));
    }
    for (int64_t v = 0; v < nv; ++v) {
        v3 s = ld3d(acc, v);
        double l = norm(s);
        if (l > 0) { st3d(n_out, v, scl(s, 1.0 / l)); if (valid_out) valid_out[v] = 1; }
        else { st3d(n_out, v, mk(0, 0, 0)); if (valid_out) valid_out[v] = 0; }
    }
    free(acc);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Per-face tangent frame and UV reliability (Sec. 6.4: tangent/bitangent in */
/* the G-buffer; UV-reliability filter)                                      */
/* ------------------------------------------------------------------------ */

static void snap(const float *UV, int64_t f, int k, int32_t res, int64_t *X, int64_t *Y) {
    double s = (double)res * 256.0;
    *X = (int64_t)nearbyint((double)UV[6 * f + 2 * k] * s);
    *Y = (int64_t)nearbyint((double)UV[6 * f + 2 * k + 1] * s);
}

/* T_f = sgn(det) (e1 dv2 - e2 dv1), B_f = sgn(det) (e2 du1 - e1 du2) with the
 * snapped integer UV deltas (du, dv) and 3D edges e1 = V1-V0, e2 = V2-V0;
 * h_f = -1 if ((e1 x e2) x T_f) . B_f < 0 else +1.
 * reliable = det != 0, e1 x e2 != 0 and all three vertex normals defined. */
int orc_face_frames(const float *V, int64_t nv, const int32_t *F, int64_t nf,
                    const float *UV, int32_t res, const uint8_t *vn_valid,
                    double *T_out, double *B_out, int8_t *h_out, uint8_t *reliable_out) {
    if (!V || !F || !UV || nv < 0 || nf < 0 || res <= 0) return ORC_EINVAL;
    for (int64_t f = 0; f < nf; ++f) {
        int64_t X[3], Y[3];
        for (int k = 0; k < 3; ++k) snap(UV, f, k, res, &X[k], &Y[k]);
        int64_t du1 = X[1] - X[0], dv1 = Y[1] - Y[0], du2 = X[2] - X[0], dv2 = Y[2] - Y[0];
        int64_t det = du1 * dv2 - du2 * dv1;
        double sg = det > 0 ? 1.0 : (det < 0 ? -1.0 : 0.0);
        v3 A = ld3f(V, F[3 * f]), B = ld3f(V, F[3 * f + 1]), C = ld3f(V, F[3 * f + 2]);
        v3 e1 = sub(B, A), e2 = sub(C, A);
        v3 T = scl(sub(scl(e1, (double)dv2), scl(e2, (double)dv1)), sg);
        v3 Bt = scl(sub(scl(e2, (double)du1), scl(e1, (double)du2)), sg);
        v3 n = cross(e1, e2);
        double hs = dot(cross(n, T), Bt);
        int ok = det != 0 && (n.x != 0 || n.y != 0 || n.z != 0);
        if (vn_valid) ok = ok && vn_valid[F[3 * f]] && vn_valid[F[3 * f + 1]] && vn_valid[F[3 * f + 2]];
        if (T_out) st3d(T_out, f, T);
        if (B_out) st3d(B_out, f, Bt);
        if (h_out) h_out[f] = hs < 0 ? -1 : 1;
        if (reliable_out) reliable_out[f] = (uint8_t)ok;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* UV-space rasterisation (G-buffer, Sec. 6.4)                               */
/* ------------------------------------------------------------------------ */

/* face_out[res*res]: covering face or -1; bary_out[res*res*3]: E_k / sum E.
 * Faces are visited in ascending order and a texel keeps its first cover, so
 * the lowest face index wins an overlap. */
int orc_raster(const float *UV, int64_t nf, int32_t res, int32_t *face_out, double *bary_out) {
    if (!UV || !face_out || nf < 0 || res <= 0) return ORC_EINVAL;
    int64_t ntex = (int64_t)res * res;
    for (int64_t t = 0; t < ntex; ++t) {
        face_out[t] = -1;
        if (bary_out) { bary_out[3 * t] = bary_out[3 * t + 1] = bary_out[3 * t + 2] = 0; }
    }
    for (int64_t f = 0; f < nf; ++f) {
        int64_t X[3], Y[3];
        for (int k = 0; k < 3; ++k) snap(UV, f, k, res, &X[k], &Y[k]);
        int64_t xmin = X[0], xmax = X[0], ymin = Y[0], ymax = Y[0];
        for (int k = 1; k < 3; ++k) {
            if (X[k] < xmin) xmin = X[k];
            if (X[k] > xmax) xmax = X[k];
            if (Y[k] < ymin) ymin = Y[k];
            if (Y[k] > ymax) ymax = Y[k];
        }
        /* texel centres 256 j + 128 within [xmin, xmax] */
        int64_t j0 = floordiv(xmin - 128 + 255, 256), j1 = floordiv(xmax - 128, 256);
        int64_t i0 = floordiv(ymin - 128 + 255, 256), i1 = floordiv(ymax - 128, 256);
        if (j0 < 0) j0 = 0;
        if (i0 < 0) i0 = 0;
        if (j1 > res - 1) j1 = res - 1;
        if (i1 > res - 1) i1 = res - 1;
        for (int64_t i = i0; i <= i1; ++i) {
            for (int64_t j = j0; j <= j1; ++j) {
                int64_t cx = 256 * j + 128, cy = 256 * i + 128;
                /* E_k: edge function of the edge opposite corner k */
                int64_t E0 = (X[2] - X[1]) * (cy - Y[1]) - (Y[2] - Y[1]) * (cx - X[1]);
                int64_t E1 = (X[0] - X[2]) * (cy - Y[2]) - (Y[0] - Y[2]) * (cx - X[2]);
                int64_t E2 = (X[1] - X[0]) * (cy - Y[0]) - (Y[1] - Y[0]) * (cx - X[0]);
                int64_t S = E0 + E1 + E2;
                int in = (E0 >= 0 && E1 >= 0 && E2 >= 0) || (E0 <= 0 && E1 <= 0 && E2 <= 0);
                if (!in || S == 0) continue;
                int64_t t = i * res + j;
                if (face_out[t] >= 0) continue;
                face_out[t] = (int32_t)f;
                if (bary_out) {
                    bary_out[3 * t] = (double)E0 / (double)S;
                    bary_out[3 * t + 1] = (double)E1 / (double)S;
                    bary_out[3 * t + 2] = (double)E2 / (double)S;
                }
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Rays: world position and interpolated smooth normal per covered texel     */
/* ------------------------------------------------------------------------ */

/* For texel list (face, b0, b1, b2): p = sum b_k V_k, m = sum b_k n_k,
 * d = m / |m|.  ok_out = 0 where |m| = 0. */
int orc_rays(const float *V, const int32_t *F, const double *vn, int64_t n,
             const int32_t *face, const double *bary, double *p_out, double *d_out, uint8_t *ok_out) {
    for (int64_t r = 0; r < n; ++r) {
        int32_t f = face[r];
        v3 p = mk(0, 0, 0), m = mk(0, 0, 0);
        for (int k = 0; k < 3; ++k) {
            int32_t v = F[3 * f + k];
            double b = bary[3 * r + k];
            p = add(p, scl(ld3f(V, v), b));
            m = add(m, scl(ld3d(vn, v), b));
        }
        double l = norm(m);
        st3d(p_out, r, p);
        if (l > 0) { st3d(d_out, r, scl(m, 1.0 / l)); ok_out[r] = 1; }
        else { st3d(d_out, r, mk(0, 0, 0)); ok_out[r] = 0; }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* High-poly correspondence: two-sided line / triangle test                 */
/* ------------------------------------------------------------------------ */

/* Signed volume s(a,b) = d . ((a-p) x (b-p)), always evaluated with the lower
 * vertex index first and negated for the reversed direction, so two faces that
 * share an edge see exactly opposite values (watertight in FP64). */
static double svol(v3 p, v3 d, const float *V, int32_t ia, int32_t ib) {
    if (ia <= ib) return dot(d, cross(sub(ld3f(V, ia), p), sub(ld3f(V, ib), p)));
    return -dot(d, cross(sub(ld3f(V, ib), p), sub(ld3f(V, ia), p)));
}

/* Line p + t d against triangle g.  With the three volumes s_k and their sum
 * S != 0, the plane crossing has barycentric weights beta = (s_bc, s_ca,
 * s_ab) / S.  RULE_PLAIN: hit iff the volumes share a sign (zeros allowed, not
 * all zero), i.e. every weight >= 0; RULE_ROBUST: hit iff every weight is >=
 * -EDGE_EPS.  q = sum beta_k v_k, t = (q - p) . d.  Returns 1 on a hit. */
static int tri_hit(v3 p, v3 d, const float *V, const int32_t *F, int64_t g, int rule, double *t,
                   double beta[3]) {
    int32_t a = F[3 * g], b = F[3 * g + 1], c = F[3 * g + 2];
    double s0 = svol(p, d, V, b, c), s1 = svol(p, d, V, c, a), s2 = svol(p, d, V, a, b);
    double S = s0 + s1 + s2;
    if (rule == RULE_PLAIN) {
        int same = (s0 >= 0 && s1 >= 0 && s2 >= 0) || (s0 <= 0 && s1 <= 0 && s2 <= 0);
        if (!same || S == 0) return 0;
    } else if (S == 0) {
        return 0;
    }
    beta[0] = s0 / S; beta[1] = s1 / S; beta[2] = s2 / S;
    if (rule != RULE_PLAIN && (beta[0] < -EDGE_EPS || beta[1] < -EDGE_EPS || beta[2] < -EDGE_EPS)) return 0;
    v3 q = add(add(scl(ld3f(V, a), beta[0]), scl(ld3f(V, b), beta[1])), scl(ld3f(V, c), beta[2]));
    *t = dot(sub(q, p), d);
    return 1;
}

/* Distance key of the robust rule: floor(|t| / w) with w = max_dist * 2^-T_QUANT_BITS. */
static int64_t tkey(double t, double max_dist) {
    return (int64_t)floor(fabs(t) * ldexp(1.0, T_QUANT_BITS) / max_dist);
}

/* (key, g) lexicographic order: is (ta, ga) better than (tb, gb)? */
static int better(double ta, int64_t ga, double tb, int64_t gb, double max_dist) {
    int64_t a = tkey(ta, max_dist), b = tkey(tb, max_dist);
    return a < b || (a == b && ga < gb);
}

/* The order of the rule: (|t|, g) for RULE_PLAIN, (key, g) for RULE_ROBUST. */
static int better_rule(int rule, double ta, int64_t ga, double tb, int64_t gb, double max_dist) {
    if (rule == RULE_PLAIN) return fabs(ta) < fabs(tb) || (fabs(ta) == fabs(tb) && ga < gb);
    return better(ta, ga, tb, gb, max_dist);
}

/* Is triangle g excluded for ray r?  exclude: [n][N_EXCLUDE] triangle ids
 * (-1: none) that the query skips (the comparator's runner-up queries), or
 * NULL. */
#define N_EXCLUDE 4
static int excluded(const int32_t *exclude, int64_t r, int64_t g) {
    if (!exclude) return 0;
    for (int k = 0; k < N_EXCLUDE; ++k)
        if (exclude[N_EXCLUDE * r + k] == g) return 1;
    return 0;
}

static int rule_ok(int rule) { return rule == RULE_PLAIN || rule == RULE_ROBUST; }

/* Brute force over every triangle in ascending index order. */
int orc_query_brute(const float *V, const int32_t *F, int64_t nf, int64_t n, const double *P,
                    const double *D, const uint8_t *active, double max_dist, int rule,
                    const int32_t *exclude, int32_t *id_out, double *t_out, double *beta_out) {
    if (!rule_ok(rule)) return ORC_EINVAL;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < n; ++r) {
        int32_t best = -1;
        double bt = 0, bb[3] = {0, 0, 0};
        if (!active || active[r]) {
            v3 p = ld3d(P, r), d = ld3d(D, r);
            for (int64_t g = 0; g < nf; ++g) {
                double t, beta[3];
                if (excluded(exclude, r, g)) continue;
                if (!tri_hit(p, d, V, F, g, rule, &t, beta)) continue;
                if (fabs(t) > max_dist) continue;
                if (best < 0 || better_rule(rule, t, g, bt, best, max_dist)) {
                    best = (int32_t)g; bt = t; bb[0] = beta[0]; bb[1] = beta[1]; bb[2] = beta[2];
                }
            }
        }
        id_out[r] = best;
        if (t_out) t_out[r] = best >= 0 ? bt : 0;
        if (beta_out) { beta_out[3 * r] = bb[0]; beta_out[3 * r + 1] = bb[1]; beta_out[3 * r + 2] = bb[2]; }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Independent FP64 BVH (median split on the longest centroid axis)          */
/* ------------------------------------------------------------------------ */

typedef struct {
    double lo[3], hi[3];
    int64_t left, right;   /* children, or -1 for a leaf */
    int64_t first, count;  /* triangle range in perm for a leaf */
} bnode;

typedef struct {
    bnode *nodes;
    int64_t nnodes;
    int64_t *perm;
} bvh;

static double *g_cent; /* centroid array used by the comparator below */
static int g_axis;
static int cmp_cent(const void *a, const void *b) {
    int64_t ia = *(const int64_t *)a, ib = *(const int64_t *)b;
    double ca = g_cent[3 * ia + g_axis], cb = g_cent[3 * ib + g_axis];
    if (ca < cb) return -1;
    if (ca > cb) return 1;
    return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

static int64_t build_rec(bvh *B, const float *V, const int32_t *F, double *cent,
                         int64_t first, int64_t count) {
    int64_t me = B->nnodes++;
    bnode *nd = &B->nodes[me];
    for (int k = 0; k < 3; ++k) { nd->lo[k] = INFINITY; nd->hi[k] = -INFINITY; }
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = first; i < first + count; ++i) {
        int64_t g = B->perm[i];
        for (int c = 0; c < 3; ++c) {
            int32_t v = F[3 * g + c];
            for (int k = 0; k < 3; ++k) {
                double x = V[3 * v + k];
                if (x < nd->lo[k]) nd->lo[k] = x;
                if (x > nd->hi[k]) nd->hi[k] = x;
            }
        }
        for (int k = 0; k < 3; ++k) {
            double x = cent[3 * g + k];
            if (x < clo[k]) clo[k] = x;
            if (x > chi[k]) chi[k] = x;
        }
    }
    /* pad outward so the box test can never reject a triangle the triangle
     * test would accept: with weights >= -EDGE_EPS the crossing lies in the
     * triangle scaled by (1 + 3 EDGE_EPS) about its centroid */
    for (int k = 0; k < 3; ++k) {
        double pad = 3.0 * EDGE_EPS * (nd->hi[k] - nd->lo[k]) + 1e-9 * (1.0 + fabs(nd->lo[k]) + fabs(nd->hi[k]));
        nd->lo[k] -= pad;
        nd->hi[k] += pad;
    }
    if (count <= 4) {
        nd->left = nd->right = -1;
        nd->first = first;
        nd->count = count;
        return me;
    }
    int axis = 0;
    double ext = chi[0] - clo[0];
    for (int k = 1; k < 3; ++k) if (chi[k] - clo[k] > ext) { ext = chi[k] - clo[k]; axis = k; }
    g_cent = cent;
    g_axis = axis;
    qsort(B->perm + first, (size_t)count, sizeof(int64_t), cmp_cent);
    int64_t half = count / 2;
    int64_t l = build_rec(B, V, F, cent, first, half);
    int64_t r = build_rec(B, V, F, cent, first + half, count - half);
    nd = &B->nodes[me];
    nd->left = l;
    nd->right = r;
    nd->first = nd->count = 0;
    return me;
}

/* Interval of line parameters t for which p + t d lies in the box, widened
 * outward by a relative 1e-12.  Returns 0 if empty. */
static int box_interval(const bnode *nd, v3 p, v3 d, double *t0, double *t1) {
    double lo = -INFINITY, hi = INFINITY;
    double pp[3] = {p.x, p.y, p.z}, dd[3] = {d.x, d.y, d.z};
    for (int k = 0; k < 3; ++k) {
        if (dd[k] == 0) {
            if (pp[k] < nd->lo[k] || pp[k] > nd->hi[k]) return 0;
            continue;
        }
        double a = (nd->lo[k] - pp[k]) / dd[k], b = (nd->hi[k] - pp[k]) / dd[k];
        double mn = a < b ? a : b, mx = a < b ? b : a;
        mn -= 1e-12 * fabs(mn);
        mx += 1e-12 * fabs(mx);
        if (mn > lo) lo = mn;
        if (mx < hi) hi = mx;
    }
    if (lo > hi) return 0;
    *t0 = lo;
    *t1 = hi;
    return 1;
}

static int32_t bvh_query(const bvh *B, const float *V, const int32_t *F, v3 p, v3 d, double max_dist,
                         int rule, const int32_t *exclude, int64_t r, double *t_out, double beta_out[3]) {
    int64_t stack[256];
    int sp = 0;
    stack[sp++] = 0;
    int32_t best = -1;
    double bt = 0, bound = max_dist * (1.0 + 1e-12);
    const double w = max_dist * ldexp(1.0, -T_QUANT_BITS);
    while (sp > 0) {
        const bnode *nd = &B->nodes[stack[--sp]];
        double t0, t1;
        if (!box_interval(nd, p, d, &t0, &t1)) continue;
        if (t0 > bound || t1 < -bound) continue; /* a node that may hold an equal or better hit is visited */
        if (nd->left < 0) {
            for (int64_t i = nd->first; i < nd->first + nd->count; ++i) {
                int64_t g = B->perm[i];
                double t, beta[3];
                if (excluded(exclude, r, g)) continue;
                if (!tri_hit(p, d, V, F, g, rule, &t, beta)) continue;
                if (fabs(t) > max_dist) continue;
                if (best < 0 || better_rule(rule, t, g, bt, best, max_dist)) {
                    best = (int32_t)g; bt = t;
                    beta_out[0] = beta[0]; beta_out[1] = beta[1]; beta_out[2] = beta[2];
                    /* plain: |t| itself; robust: the upper end of the best key's bin; widened */
                    bound = (rule == RULE_PLAIN ? fabs(t) : (double)(tkey(t, max_dist) + 1) * w) * (1.0 + 1e-12);
                }
            }
        } else {
            if (sp + 2 > 256) return -100; /* cannot happen for median splits of < 2^60 tris */
            stack[sp++] = nd->right;
            stack[sp++] = nd->left;
        }
    }
    *t_out = bt;
    return best;
}

static void bvh_make(bvh *B, const float *V, const int32_t *F, int64_t nf) {
    B->nodes = (bnode *)malloc(sizeof(bnode) * (size_t)(2 * (nf > 0 ? nf : 1)));
    B->perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nf > 0 ? nf : 1));
    B->nnodes = 0;
    double *cent = (double *)malloc(sizeof(double) * (size_t)(3 * (nf > 0 ? nf : 1)));
    for (int64_t g = 0; g < nf; ++g) {
        B->perm[g] = g;
        for (int k = 0; k < 3; ++k)
            cent[3 * g + k] = ((double)V[3 * F[3 * g] + k] + V[3 * F[3 * g + 1] + k] + V[3 * F[3 * g + 2] + k]) / 3.0;
    }
    if (nf > 0) build_rec(B, V, F, cent, 0, nf);
    free(cent);
}

static void bvh_release(bvh *B) {
    free(B->perm);
    free(B->nodes);
}

int orc_query_bvh(const float *V, int64_t nv, const int32_t *F, int64_t nf, int64_t n, const double *P,
                  const double *D, const uint8_t *active, double max_dist, int rule,
                  const int32_t *exclude, int32_t *id_out, double *t_out, double *beta_out) {
    (void)nv;
    if (!rule_ok(rule)) return ORC_EINVAL;
    bvh B;
    bvh_make(&B, V, F, nf);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : err)
    for (int64_t r = 0; r < n; ++r) {
        double t = 0, beta[3] = {0, 0, 0};
        int32_t id = -1;
        if ((!active || active[r]) && nf > 0) {
            id = bvh_query(&B, V, F, ld3d(P, r), ld3d(D, r), max_dist, rule, exclude, r, &t, beta);
            if (id == -100) { err = 1; id = -1; }
        }
        id_out[r] = id;
        if (t_out) t_out[r] = id >= 0 ? t : 0;
        if (beta_out) { beta_out[3 * r] = beta[0]; beta_out[3 * r + 1] = beta[1]; beta_out[3 * r + 2] = beta[2]; }
    }
    bvh_release(&B);
    return err ? ORC_EINVAL : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Closest-point query (the paper's own form of the correspondence step)     */
/* ------------------------------------------------------------------------ */
/*
 * Sec. 6.4 locates, for each texel's world position p, the closest point of
 * the high-poly surface and rejects it when it is farther than a distance
 * bound (the paper: 1% of the bounding-box diagonal; here max_dist).  Per
 * triangle the nearest point q minimises |p - q| over the triangle: the
 * orthogonal projection of p onto the plane when its barycentric weights are
 * all >= 0; otherwise the minimum lies on the border (a convex function over a
 * convex set whose free minimum is outside), i.e. the nearest of the three
 * edges' nearest points.  Over the mesh the winner minimises
 * (floor(dist / w), index) with w = max_dist 2^-20, as for the ray query, so a
 * closest point on a shared edge or vertex resolves to the lower index.
 */

/* Parameter in [0, 1] of the point of segment [a, b] nearest to p. */
static double seg_param(v3 p, v3 a, v3 b) {
    v3 ab = sub(b, a);
    double l2 = dot(ab, ab);
    if (!(l2 > 0)) return 0.0;
    double s = dot(sub(p, a), ab) / l2;
    return s < 0 ? 0.0 : (s > 1 ? 1.0 : s);
}

/* Distance from p to triangle g and the barycentric weights of its nearest point. */
static double tri_closest(v3 p, const float *V, const int32_t *F, int64_t g, double w[3]) {
    v3 P3[3];
    for (int k = 0; k < 3; ++k) P3[k] = ld3f(V, F[3 * g + k]);
    v3 n = cross(sub(P3[1], P3[0]), sub(P3[2], P3[0]));
    double nn = dot(n, n);
    if (nn > 0) {
        v3 q = sub(p, scl(n, dot(n, sub(p, P3[0])) / nn));
        double wa = dot(n, cross(sub(P3[1], q), sub(P3[2], q))) / nn;
        double wb = dot(n, cross(sub(P3[2], q), sub(P3[0], q))) / nn;
        double wc = dot(n, cross(sub(P3[0], q), sub(P3[1], q))) / nn;
        if (wa >= 0 && wb >= 0 && wc >= 0) {
            w[0] = wa; w[1] = wb; w[2] = wc;
            return norm(sub(p, q));
        }
    }
    double best = INFINITY;
    for (int e = 0; e < 3; ++e) {
        int i = e, j = (e + 1) % 3;
        double s = seg_param(p, P3[i], P3[j]);
        double dd = norm(sub(p, add(P3[i], scl(sub(P3[j], P3[i]), s))));
        if (dd < best) {
            best = dd;
            w[0] = w[1] = w[2] = 0;
            w[i] = 1 - s;
            w[j] = s;
        }
    }
    return best;
}

/* Brute force over every triangle in ascending index order. */
int orc_closest_brute(const float *V, const int32_t *F, int64_t nf, int64_t n, const double *P,
                      const uint8_t *active, double max_dist, int32_t *id_out, double *dist_out,
                      double *w_out) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < n; ++r) {
        int32_t best = -1;
        double bd = 0, bw[3] = {0, 0, 0};
        if (!active || active[r]) {
            v3 p = ld3d(P, r);
            for (int64_t g = 0; g < nf; ++g) {
                double w[3];
                double dd = tri_closest(p, V, F, g, w);
                if (!(dd <= max_dist)) continue;
                if (best < 0 || better(dd, g, bd, best, max_dist)) {
                    best = (int32_t)g; bd = dd; bw[0] = w[0]; bw[1] = w[1]; bw[2] = w[2];
                }
            }
        }
        id_out[r] = best;
        if (dist_out) dist_out[r] = best >= 0 ? bd : 0;
        if (w_out) { w_out[3 * r] = bw[0]; w_out[3 * r + 1] = bw[1]; w_out[3 * r + 2] = bw[2]; }
    }
    return ORC_OK;
}

/* Distance from p to the box (0 inside). */
static double box_dist(const bnode *nd, v3 p) {
    double pp[3] = {p.x, p.y, p.z}, s = 0;
    for (int k = 0; k < 3; ++k) {
        double e = 0;
        if (pp[k] < nd->lo[k]) e = nd->lo[k] - pp[k];
        else if (pp[k] > nd->hi[k]) e = pp[k] - nd->hi[k];
        s += e * e;
    }
    return sqrt(s);
}

/* The same query on the FP64 BVH: nodes farther than the current best key's
 * bin are skipped (boxes are padded outward, and the bound has a relative
 * margin), so the result equals the brute force. */
static int32_t bvh_closest(const bvh *B, const float *V, const int32_t *F, v3 p, double max_dist,
                           double *d_out, double w_out[3]) {
    int64_t stack[256];
    int sp = 0;
    int32_t best = -1;
    double bd = 0, bw[3] = {0, 0, 0};
    double bound = max_dist;
    stack[sp++] = 0;
    while (sp > 0) {
        const bnode *nd = &B->nodes[stack[--sp]];
        if (box_dist(nd, p) > bound * (1 + 1e-12)) continue;
        if (nd->left < 0) {
            for (int64_t i = nd->first; i < nd->first + nd->count; ++i) {
                int64_t g = B->perm[i];
                double w[3];
                double dd = tri_closest(p, V, F, g, w);
                if (!(dd <= max_dist)) continue;
                if (best < 0 || better(dd, g, bd, best, max_dist)) {
                    best = (int32_t)g; bd = dd; bw[0] = w[0]; bw[1] = w[1]; bw[2] = w[2];
                    bound = (double)(tkey(bd, max_dist) + 1) * ldexp(max_dist, -T_QUANT_BITS);
                }
            }
            continue;
        }
        if (sp + 2 > 256) return -100;
        /* the nearer child is popped first, so the bound tightens early */
        int64_t near = nd->left, far = nd->right;
        if (box_dist(&B->nodes[far], p) < box_dist(&B->nodes[near], p)) { near = nd->right; far = nd->left; }
        stack[sp++] = far;
        stack[sp++] = near;
    }
    *d_out = bd;
    w_out[0] = bw[0]; w_out[1] = bw[1]; w_out[2] = bw[2];
    return best;
}

int orc_closest_bvh(const float *V, const int32_t *F, int64_t nf, int64_t n, const double *P,
                    const uint8_t *active, double max_dist, int32_t *id_out, double *dist_out,
                    double *w_out) {
    bvh B;
    bvh_make(&B, V, F, nf);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : err)
    for (int64_t r = 0; r < n; ++r) {
        double dd = 0, w[3] = {0, 0, 0};
        int32_t id = -1;
        if ((!active || active[r]) && nf > 0) {
            id = bvh_closest(&B, V, F, ld3d(P, r), max_dist, &dd, w);
            if (id == -100) { err = 1; id = -1; }
        }
        id_out[r] = id;
        if (dist_out) dist_out[r] = id >= 0 ? dd : 0;
        if (w_out) { w_out[3 * r] = w[0]; w_out[3 * r + 1] = w[1]; w_out[3 * r + 2] = w[2]; }
    }
    bvh_release(&B);
    return err ? ORC_EINVAL : ORC_OK;
}

/* Near ties of the closest-point query: near_out[r] = 1 when some triangle
 * other than the winner id[r] lies at a distance within delta of the winner's
 * dist[r] but differs from it by more than eps_exact (triangles sharing the
 * nearest vertex or edge are at the same distance: exact ties, which both
 * sides resolve to the lower index).  An FP32 evaluation of the distances may
 * order such a near tie either way.  On the FP64 BVH. */
int orc_closest_near(const float *V, const int32_t *F, int64_t nf, int64_t n, const double *P,
                     const int32_t *id, const double *dist, double delta, double eps_exact,
                     uint8_t *near_out) {
    bvh B;
    bvh_make(&B, V, F, nf);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : err)
    for (int64_t r = 0; r < n; ++r) {
        near_out[r] = 0;
        if (id[r] < 0 || nf == 0) continue;
        v3 p = ld3d(P, r);
        const double lim = dist[r] + delta;
        int64_t stack[256];
        int sp = 0;
        stack[sp++] = 0;
        while (sp > 0 && !near_out[r]) {
            const bnode *nd = &B.nodes[stack[--sp]];
            if (box_dist(nd, p) > lim * (1 + 1e-12)) continue;
            if (nd->left < 0) {
                for (int64_t i = nd->first; i < nd->first + nd->count; ++i) {
                    int64_t g = B.perm[i];
                    if (g == id[r]) continue;
                    double w[3];
                    double dd = tri_closest(p, V, F, g, w);
                    if (fabs(dd - dist[r]) <= delta && fabs(dd - dist[r]) > eps_exact) { near_out[r] = 1; break; }
                }
                continue;
            }
            if (sp + 2 > 256) { err = 1; break; }
            stack[sp++] = nd->right;
            stack[sp++] = nd->left;
        }
    }
    bvh_release(&B);
    return err ? ORC_EINVAL : ORC_OK;
}

/* Comparator support: distance from P[r] to a given triangle g[r]. */
int orc_closest_check(const float *V, const int32_t *F, int64_t n, const double *P, const int32_t *g,
                      double *dist_out) {
    for (int64_t r = 0; r < n; ++r) {
        double w[3];
        dist_out[r] = tri_closest(ld3d(P, r), V, F, g[r], w);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Hidden-face removal (Sec. 6.2): visibility rays from viewpoints around    */
/* the mesh, then a flood fill over shared edges gated by the face normals   */
/* ------------------------------------------------------------------------ */
/*
 * Readings (the paper names the viewpoint count, the resolution and the
 * rule, not the camera):
 *   view v: a pinhole at eye_v looking at `target` (both float); forward f =
 *     (target - eye) / |target - eye|; helper axis a = the world axis with the
 *     smallest |target_k - eye_k| (the lowest k on ties; the differences of
 *     float inputs are exact); right r = (f x a) / |f x a|; up u = r x f;
 *   pixel (i, j) of a res x res image: x = ((j + 1/2) 2 / res - 1) tan_half,
 *     y = (1 - (i + 1/2) 2 / res) tan_half; the ray leaves the eye along
 *     normalise(f + x r + y u);
 *   first hit: the hit rule of the bake (edge tolerance EDGE_EPS) on the
 *     half-line, t in (0, t_far], winner minimising (floor(t / w), index) with
 *     w = t_far 2^-20; a face is visible when it is some ray's first hit;
 *   flood fill: faces f and g are adjacent when they share two distinct vertex
 *     indices; g joins the exterior from an exterior neighbour f when
 *     n_f . n_g > 0, n = (V1 - V0) x (V2 - V0) evaluated in FP64 from the
 *     float vertices in this order (x, y, z; no fused operations); seeds are
 *     the visible faces.  The condition is symmetric, so the exterior is the
 *     set of faces connected to a seed through such edges, whatever the order
 *     of the traversal.
 */

/* Camera frame of view v: forward, right, up.  The helper axis is chosen on
 * the differences target - eye themselves (exact for float inputs), so the
 * choice does not depend on how the forward vector is rounded. */
static int camera_frame(const float *eyes, const double *target, int64_t v, v3 *f_out, v3 *r_out, v3 *u_out) {
    v3 e = ld3f(eyes, v), c = mk(target[0], target[1], target[2]);
    v3 f = sub(c, e);
    double af[3] = {fabs(f.x), fabs(f.y), fabs(f.z)};
    double lf = norm(f);
    if (!(lf > 0)) return ORC_EINVAL;
    f = scl(f, 1.0 / lf);
    int k = 0;
    if (af[1] < af[k]) k = 1;
    if (af[2] < af[k]) k = 2;
    v3 a = mk(k == 0, k == 1, k == 2);
    v3 r = cross(f, a);
    r = scl(r, 1.0 / norm(r));
    *f_out = f;
    *r_out = r;
    *u_out = cross(r, f);
    return ORC_OK;
}

/* Ray q = (v res + i) res + j: origin eye_v, unit direction of pixel (i, j). */
static int camera_ray(const float *eyes, const double *target, double tan_half, int32_t res, int64_t q,
                      v3 *p_out, v3 *d_out) {
    int64_t v = q / ((int64_t)res * res), pix = q % ((int64_t)res * res);
    int64_t i = pix / res, j = pix % res;
    v3 e = ld3f(eyes, v), f, r, u;
    if (camera_frame(eyes, target, v, &f, &r, &u)) return ORC_EINVAL;
    double x = ((j + 0.5) * 2.0 / res - 1.0) * tan_half;
    double y = (1.0 - (i + 0.5) * 2.0 / res) * tan_half;
    v3 d = add(add(f, scl(r, x)), scl(u, y));
    *p_out = e;
    *d_out = scl(d, 1.0 / norm(d));
    return ORC_OK;
}

/* Rays of every pixel of every view, ray index (v res + i) res + j. */
int orc_camera_rays(const float *eyes, int32_t nviews, const double *target, double tan_half, int32_t res,
                    double *P_out, double *D_out) {
    const int64_t n = (int64_t)nviews * res * res;
    for (int64_t q = 0; q < n; ++q) {
        v3 p, d;
        if (camera_ray(eyes, target, tan_half, res, q, &p, &d)) return ORC_EINVAL;
        st3d(P_out, q, p);
        st3d(D_out, q, d);
    }
    return ORC_OK;
}

/* The rays of a list of ray indices. */
int orc_camera_rays_at(const float *eyes, const double *target, double tan_half, int32_t res, int64_t n,
                       const int64_t *which, double *P_out, double *D_out) {
    for (int64_t k = 0; k < n; ++k) {
        v3 p, d;
        if (camera_ray(eyes, target, tan_half, res, which[k], &p, &d)) return ORC_EINVAL;
        st3d(P_out, k, p);
        st3d(D_out, k, d);
    }
    return ORC_OK;
}

/* First hit of each half-line by brute force over every triangle, under
 * `rule` (the order is then on t > 0 itself); `exclude` as for the line query. */
int orc_first_hit_brute(const float *V, const int32_t *F, int64_t nf, int64_t n, const double *P,
                        const double *D, double t_far, int rule, const int32_t *exclude,
                        int32_t *id_out, double *t_out) {
    if (!rule_ok(rule)) return ORC_EINVAL;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < n; ++r) {
        int32_t best = -1;
        double bt = 0;
        v3 p = ld3d(P, r), d = ld3d(D, r);
        for (int64_t g = 0; g < nf; ++g) {
            double t, beta[3];
            if (excluded(exclude, r, g)) continue;
            if (!tri_hit(p, d, V, F, g, rule, &t, beta)) continue;
            if (!(t > 0) || t > t_far) continue;
            if (best < 0 || better_rule(rule, t, g, bt, best, t_far)) { best = (int32_t)g; bt = t; }
        }
        id_out[r] = best;
        if (t_out) t_out[r] = best >= 0 ? bt : 0;
    }
    return ORC_OK;
}

/* The same on the FP64 BVH: a node is skipped when its interval ends before
 * t = 0 or starts past the best hit (plain) or the upper end of the best
 * key's bin (robust). */
static int32_t bvh_first_hit(const bvh *B, const float *V, const int32_t *F, v3 p, v3 d, double t_far,
                             int rule, const int32_t *exclude, int64_t r, double *t_out) {
    int64_t stack[256];
    int sp = 0;
    stack[sp++] = 0;
    int32_t best = -1;
    double bt = 0, bound = t_far * (1.0 + 1e-12);
    const double w = t_far * ldexp(1.0, -T_QUANT_BITS);
    while (sp > 0) {
        const bnode *nd = &B->nodes[stack[--sp]];
        double t0, t1;
        if (!box_interval(nd, p, d, &t0, &t1)) continue;
        if (t0 > bound || t1 < 0) continue;
        if (nd->left < 0) {
            for (int64_t i = nd->first; i < nd->first + nd->count; ++i) {
                int64_t g = B->perm[i];
                double t, beta[3];
                if (excluded(exclude, r, g)) continue;
                if (!tri_hit(p, d, V, F, g, rule, &t, beta)) continue;
                if (!(t > 0) || t > t_far) continue;
                if (best < 0 || better_rule(rule, t, g, bt, best, t_far)) {
                    best = (int32_t)g; bt = t;
                    bound = (rule == RULE_PLAIN ? t : (double)(tkey(t, t_far) + 1) * w) * (1.0 + 1e-12);
                }
            }
        } else {
            if (sp + 2 > 256) return -100;
            stack[sp++] = nd->right;
            stack[sp++] = nd->left;
        }
    }
    *t_out = bt;
    return best;
}

int orc_first_hit_bvh(const float *V, const int32_t *F, int64_t nf, int64_t n, const double *P, const double *D,
                      double t_far, int rule, const int32_t *exclude, int32_t *id_out, double *t_out) {
    if (!rule_ok(rule)) return ORC_EINVAL;
    bvh B;
    bvh_make(&B, V, F, nf);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(| : err)
    for (int64_t r = 0; r < n; ++r) {
        double t = 0;
        int32_t id = -1;
        if (nf > 0) {
            id = bvh_first_hit(&B, V, F, ld3d(P, r), ld3d(D, r), t_far, rule, exclude, r, &t);
            if (id == -100) { err = 1; id = -1; }
        }
        id_out[r] = id;
        if (t_out) t_out[r] = id >= 0 ? t : 0;
    }
    bvh_release(&B);
    return err ? ORC_EINVAL : ORC_OK;
}

/* Unnormalised face normal (V1 - V0) x (V2 - V0) from the float vertices. */
static v3 face_normal(const float *V, const int32_t *F, int64_t f) {
    v3 a = ld3f(V, F[3 * f]), b = ld3f(V, F[3 * f + 1]), c = ld3f(V, F[3 * f + 2]);
    return cross(sub(b, a), sub(c, a));
}

/* Number of distinct vertex indices faces f and g have in common. */
static int shared_vertices(const int32_t *F, int64_t f, int64_t g) {
    int n = 0;
    for (int i = 0; i < 3; ++i) {
        int32_t x = F[3 * f + i];
        int dup = 0;
        for (int k = 0; k < i; ++k) dup |= F[3 * f + k] == x;
        if (dup) continue;
        if (F[3 * g] == x || F[3 * g + 1] == x || F[3 * g + 2] == x) ++n;
    }
    return n;
}

/* Breadth-first flood fill from the seed faces (ext_out = 1 for the seeds and
 * every face reached).  Faces are found through per-vertex face lists. */
int orc_flood_fill(const float *V, int64_t nv, const int32_t *F, int64_t nf, const uint8_t *seed,
                   uint8_t *ext_out) {
    int64_t *deg = (int64_t *)calloc((size_t)nv + 1, sizeof(int64_t));
    int64_t *lst = (int64_t *)malloc(sizeof(int64_t) * (size_t)(3 * nf + 1));
    int64_t *fill = (int64_t *)calloc((size_t)nv + 1, sizeof(int64_t));
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nf + 1));
    if (!deg || !lst || !fill || !queue) { free(deg); free(lst); free(fill); free(queue); return ORC_EINVAL; }
    for (int64_t f = 0; f < nf; ++f)
        for (int i = 0; i < 3; ++i) {
            int32_t x = F[3 * f + i];
            if (x < 0 || x >= nv) { free(deg); free(lst); free(fill); free(queue); return ORC_EINVAL; }
            int dup = 0;
            for (int k = 0; k < i; ++k) dup |= F[3 * f + k] == x;
            if (!dup) deg[x + 1]++;
        }
    for (int64_t v = 0; v < nv; ++v) deg[v + 1] += deg[v];
    for (int64_t f = 0; f < nf; ++f)
        for (int i = 0; i < 3; ++i) {
            int32_t x = F[3 * f + i];
            int dup = 0;
            for (int k = 0; k < i; ++k) dup |= F[3 * f + k] == x;
            if (!dup) lst[deg[x] + fill[x]++] = f;
        }
    int64_t head = 0, tail = 0;
    for (int64_t f = 0; f < nf; ++f) {
        ext_out[f] = seed[f] ? 1 : 0;
        if (seed[f]) queue[tail++] = f;
    }
    while (head < tail) {
        int64_t f = queue[head++];
        v3 nf_ = face_normal(V, F, f);
        for (int i = 0; i < 3; ++i) {
            int32_t x = F[3 * f + i];
            for (int64_t k = deg[x]; k < deg[x + 1]; ++k) {
                int64_t g = lst[k];
                if (g == f || ext_out[g] || shared_vertices(F, f, g) < 2) continue;
                if (dot(nf_, face_normal(V, F, g)) > 0) {
                    ext_out[g] = 1;
                    queue[tail++] = g;
                }
            }
        }
    }
    free(deg); free(lst); free(fill); free(queue);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Backprojection precompute (Sec. 7.4, TextureGen Postprocessing): per     */
/* atlas texel and view, the image position, the incidence and the depth-    */
/* buffer visibility                                                          */
/* ------------------------------------------------------------------------ */
/*
 * Readings: the texel's surface point p and unit smooth normal n are the
 * bake's G-buffer (rasterised atlas, interpolated area-weighted vertex
 * normals); the views are the pinholes of the hidden-face pass; the viewing
 * direction is d_k = (e_k - p) / |e_k - p| and the raw incidence max(0, n.d_k);
 * the depth buffer of view k holds, per pixel, the view-axis depth z = t (d.f)
 * of the pixel ray's first hit (+inf where it hits nothing), i.e. a depth
 * buffer sampled at pixel centres; with q = p - e_k and z = q.f, the texel's
 * image coordinates are col = (q.r / (z tan_half) + 1) res / 2 - 1/2 and
 * row = (1 - q.u / (z tan_half)) res / 2 - 1/2 (pixel centres at integers),
 * inside when z > 0 and both lie in [-1/2, res - 1/2); it is occluded when z
 * exceeds the depth of its nearest pixel (floor(row + 1/2), floor(col + 1/2))
 * by more than tol.  The incidence is 0 outside the image, when occluded, or
 * where n is undefined; image coordinates are (-1, -1) outside.
 */
int orc_view_maps(const double *P, const double *N, const uint8_t *ok, int64_t n, const float *eyes, int32_t nviews,
                  const double *target, double tan_half, int32_t res, const double *ray_t, double tol,
                  double *uv_out, double *inc_out) {
    const int64_t px = (int64_t)res * res;
    for (int32_t k = 0; k < nviews; ++k) {
        v3 f, r, u, e = ld3f(eyes, k);
        if (camera_frame(eyes, target, k, &f, &r, &u)) return ORC_EINVAL;
        for (int64_t t = 0; t < n; ++t) {
            double *uv = uv_out + 2 * ((int64_t)k * n + t);
            double *inc = inc_out + (int64_t)k * n + t;
            uv[0] = uv[1] = -1.0;
            *inc = 0.0;
            v3 p = ld3d(P, t), q = sub(p, e);
            double z = dot(q, f);
            if (!(z > 0)) continue;
            double col = (dot(q, r) / (z * tan_half) + 1.0) * res / 2.0 - 0.5;
            double row = (1.0 - dot(q, u) / (z * tan_half)) * res / 2.0 - 0.5;
            if (!(col >= -0.5 && col < res - 0.5 && row >= -0.5 && row < res - 0.5)) continue;
            uv[0] = col;
            uv[1] = row;
            if (!ok[t]) continue;
            int64_t i = (int64_t)floor(row + 0.5), j = (int64_t)floor(col + 0.5);
            int64_t pq = (int64_t)k * px + i * res + j;
            double zb = INFINITY;
            if (ray_t[pq] > 0) {
                v3 pe, pd;
                if (camera_ray(eyes, target, tan_half, res, pq, &pe, &pd)) return ORC_EINVAL;
                zb = ray_t[pq] * dot(pd, f);
            }
            if (z > zb + tol) continue;
            v3 dk = scl(sub(e, p), 1.0 / norm(sub(e, p)));
            double c = dot(ld3d(N, t), dk);
            *inc = c > 0 ? c : 0.0;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Encoding in the texel's tangent frame (Sec. 6.4)                          */
/* ------------------------------------------------------------------------ */

/* For each ray with hit id >= 0: h = sum beta_k N_{g_k}; n = h/|h|;
 * T' = normalise(T_f - (d.T_f) d); B' = h_f (d x T'); out = (n.T', n.B', n.d).
 * status_io holds the query result on entry (id or -1) and the final status on
 * exit; rays already marked unreliable (-2) are left as they are.  Non-hits
 * get (0,0,1). */
int orc_encode(const int32_t *hiF, const float *hiN, int64_t n, const int32_t *lo_face,
               const double *D, const double *Tf, const int8_t *hf, const double *beta,
               int32_t *status_io, double *out) {
    for (int64_t r = 0; r < n; ++r) {
        v3 o = mk(0, 0, 1);
        int32_t st = status_io[r];
        if (st >= 0) {
            v3 d = ld3d(D, r);
            int32_t f = lo_face[r];
            v3 T = ld3d(Tf, f);
            v3 Tp = sub(T, scl(d, dot(d, T)));
            double lt = norm(Tp);
            v3 h = mk(0, 0, 0);
            for (int k = 0; k < 3; ++k) h = add(h, scl(ld3f(hiN, hiF[3 * st + k]), beta[3 * r + k]));
            double lh = norm(h);
            if (lt == 0 || lh == 0) {
                st = ST_UNREL;
            } else {
                Tp = scl(Tp, 1.0 / lt);
                v3 nh = scl(h, 1.0 / lh);
                v3 Bp = scl(cross(d, Tp), (double)hf[f]);
                o = mk(dot(nh, Tp), dot(nh, Bp), dot(nh, d));
            }
        }
        status_io[r] = st;
        st3d(out, r, o);
    }
    return ORC_OK;
}

/* Tangent-frame degeneracy alone (T_f parallel to d), checked before the query. */
int orc_frame_ok(int64_t n, const int32_t *lo_face, const double *D, const double *Tf, uint8_t *ok_out) {
    for (int64_t r = 0; r < n; ++r) {
        v3 d = ld3d(D, r), T = ld3d(Tf, lo_face[r]);
        v3 Tp = sub(T, scl(d, dot(d, T)));
        ok_out[r] = norm(Tp) > 0;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Chart dilation (Sec. 6.4: dilated at UV seams against mip bleed)          */
/* ------------------------------------------------------------------------ */

/* map [res*res*3], level [res*res]: 0 = has a value before dilation, 255 =
 * empty.  Pass k (1..passes) fills each still-empty texel with the normalised
 * sum of its 8 neighbours whose level is < k; a texel with no such neighbour or
 * a zero sum stays empty.  Neighbour order: rows -1,0,+1, columns -1,0,+1. */
int orc_dilate(double *map, uint8_t *level, int32_t res, int32_t passes) {
    if (!map || !level || res <= 0 || passes < 0 || passes > 254) return ORC_EINVAL;
    for (int k = 1; k <= passes; ++k) {
        for (int64_t i = 0; i < res; ++i) {
            for (int64_t j = 0; j < res; ++j) {
                int64_t t = i * res + j;
                if (level[t] != 255) continue;
                v3 s = mk(0, 0, 0);
                int cnt = 0;
                for (int di = -1; di <= 1; ++di)
                    for (int dj = -1; dj <= 1; ++dj) {
                        if (di == 0 && dj == 0) continue;
                        int64_t ii = i + di, jj = j + dj;
                        if (ii < 0 || jj < 0 || ii >= res || jj >= res) continue;
                        int64_t u = ii * res + jj;
                        if (level[u] < k) { s = add(s, ld3d(map, u)); ++cnt; }
                    }
                if (cnt == 0) continue;
                double l = norm(s);
                if (l == 0) continue;
                st3d(map, t, scl(s, 1.0 / l));
                level[t] = (uint8_t)k;
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Comparator support: plane crossing and distance to a given triangle       */
/* ------------------------------------------------------------------------ */

/* Distance from q to segment [a, b]. */
static double seg_dist(v3 q, v3 a, v3 b) {
    v3 ab = sub(b, a);
    double l2 = dot(ab, ab);
    double s = l2 > 0 ? dot(sub(q, a), ab) / l2 : 0.0;
    if (s < 0) s = 0;
    if (s > 1) s = 1;
    return norm(sub(q, add(a, scl(ab, s))));
}

/* Distance from a point q lying in the plane of triangle (a,b,c) to the
 * triangle: 0 if the three sub-triangle orientations against the face normal
 * agree (q inside or on the border), else the nearest of the three edges. */
static double in_plane_dist(v3 q, v3 a, v3 b, v3 c) {
    v3 n = cross(sub(b, a), sub(c, a));
    double wa = dot(n, cross(sub(b, q), sub(c, q)));
    double wb = dot(n, cross(sub(c, q), sub(a, q)));
    double wc = dot(n, cross(sub(a, q), sub(b, q)));
    if ((wa >= 0 && wb >= 0 && wc >= 0) || (wa <= 0 && wb <= 0 && wc <= 0)) return 0.0;
    double d0 = seg_dist(q, a, b), d1 = seg_dist(q, b, c), d2 = seg_dist(q, c, a);
    double m = d0 < d1 ? d0 : d1;
    return m < d2 ? m : d2;
}

/* For each (ray, triangle g): t_g = line parameter where p + t d crosses g's
 * plane (NaN if parallel or degenerate), delta_g = distance of that crossing
 * point from the triangle (0 inside) and bmin_g = the smallest barycentric
 * weight of the crossing (the quantity the hit rule thresholds). */
int orc_plane_check(const float *V, const int32_t *F, int64_t n, const double *P, const double *D,
                    const int32_t *g, double *t_out, double *delta_out, double *bmin_out) {
    for (int64_t r = 0; r < n; ++r) {
        v3 p = ld3d(P, r), d = ld3d(D, r);
        v3 a = ld3f(V, F[3 * g[r]]), b = ld3f(V, F[3 * g[r] + 1]), c = ld3f(V, F[3 * g[r] + 2]);
        v3 nn = cross(sub(b, a), sub(c, a));
        double den = dot(nn, d);
        if (den == 0) { t_out[r] = NAN; delta_out[r] = INFINITY; if (bmin_out) bmin_out[r] = -INFINITY; continue; }
        double t = dot(nn, sub(a, p)) / den;
        v3 q = add(p, scl(d, t));
        t_out[r] = t;
        delta_out[r] = in_plane_dist(q, a, b, c);
        if (bmin_out) {
            int32_t ia = F[3 * g[r]], ib = F[3 * g[r] + 1], ic = F[3 * g[r] + 2];
            double s0 = svol(p, d, V, ib, ic), s1 = svol(p, d, V, ic, ia), s2 = svol(p, d, V, ia, ib);
            double S = s0 + s1 + s2;
            double m = s0 / S;
            if (s1 / S < m) m = s1 / S;
            if (s2 / S < m) m = s2 / S;
            bmin_out[r] = S != 0 ? m : -INFINITY;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Frozen-selection forward and its adjoint (backward of a map loss)         */
/* ------------------------------------------------------------------------ */
/*
 * With the texel -> low-poly face assignment, its barycentrics b, the hit
 * triangle g and the handedness h_f held fixed, each texel's output is a
 * smooth function of the low-poly positions lo_V (through p, the vertex
 * normals and T_f) and of the three high-poly normals of g:
 *   n_v = s_v/|s_v|, s_v = sum_{faces at v} (V1-V0) x (V2-V0)
 *   p = sum b_k V_k,  m = sum b_k n_k,  d = m/|m|
 *   p + t d = A + beta1 (B-A) + beta2 (C-A)      (crossing of g's plane)
 *   h = beta0 N0 + beta1 N1 + beta2 N2,  n = h/|h|
 *   T~ = T_f - (d.T_f) d, T' = T~/|T~|, B' = h_f (d x T')
 *   out = (n.T', n.B', n.d)
 * The adjoint walks the same chain backwards, in FP64, summing in ray order.
 */

static void lo_vertex_sums(const float *V, int64_t nv, const int32_t *F, int64_t nf, double *s) {
    for (int64_t i = 0; i < 3 * nv; ++i) s[i] = 0;
    for (int64_t f = 0; f < nf; ++f) {
        v3 A = ld3f(V, F[3 * f]), B = ld3f(V, F[3 * f + 1]), C = ld3f(V, F[3 * f + 2]);
        v3 c = cross(sub(B, A), sub(C, A));
        for (int k = 0; k < 3; ++k) st3d(s, F[3 * f + k], add(ld3d(s, F[3 * f + k]), c));
    }
}

/* T_f from the snapped UV deltas (same definition as orc_face_frames). */
static v3 face_tangent(const float *V, const int32_t *F, const float *UV, int32_t res, int64_t f,
                       double *c1, double *c2) {
    int64_t X[3], Y[3];
    for (int k = 0; k < 3; ++k) snap(UV, f, k, res, &X[k], &Y[k]);
    int64_t du1 = X[1] - X[0], dv1 = Y[1] - Y[0], du2 = X[2] - X[0], dv2 = Y[2] - Y[0];
    int64_t det = du1 * dv2 - du2 * dv1;
    double sg = det > 0 ? 1.0 : (det < 0 ? -1.0 : 0.0);
    /* T_f = c1 e1 + c2 e2 */
    *c1 = sg * (double)dv2;
    *c2 = -sg * (double)dv1;
    v3 A = ld3f(V, F[3 * f]), B = ld3f(V, F[3 * f + 1]), C = ld3f(V, F[3 * f + 2]);
    return add(scl(sub(B, A), *c1), scl(sub(C, A), *c2));
}

/* Solve [a | b | c] x = r by Cramer's rule. */
static v3 solve3(v3 a, v3 b, v3 c, v3 r) {
    double D = dot(a, cross(b, c));
    return mk(dot(r, cross(b, c)) / D, dot(a, cross(r, c)) / D, dot(a, cross(b, r)) / D);
}

/* Per-ray forward state shared by the frozen forward and the adjoint. */
typedef struct {
    v3 p, m, d, Tf, Tt, Tp, Bp, h, n;
    double lm, lt, lh, t, b1, b2, c1, c2;
    v3 A, e1, e2, N[3];
    int32_t lv[3], hv[3];
} rstate;

static void ray_forward(const float *loV, const int32_t *loF, const double *nrm, const float *UV,
                        int32_t res, const float *hiV, const int32_t *hiF, const float *hiN,
                        int32_t face, const double *bary, int32_t g, int8_t hf, rstate *S) {
    for (int k = 0; k < 3; ++k) { S->lv[k] = loF[3 * face + k]; S->hv[k] = hiF[3 * g + k]; }
    S->p = mk(0, 0, 0); S->m = mk(0, 0, 0);
    for (int k = 0; k < 3; ++k) {
        S->p = add(S->p, scl(ld3f(loV, S->lv[k]), bary[k]));
        S->m = add(S->m, scl(ld3d(nrm, S->lv[k]), bary[k]));
    }
    S->lm = norm(S->m);
    S->d = scl(S->m, 1.0 / S->lm);
    S->A = ld3f(hiV, S->hv[0]);
    S->e1 = sub(ld3f(hiV, S->hv[1]), S->A);
    S->e2 = sub(ld3f(hiV, S->hv[2]), S->A);
    v3 x = solve3(scl(S->d, -1.0), S->e1, S->e2, sub(S->p, S->A));
    S->t = x.x; S->b1 = x.y; S->b2 = x.z;
    double b0 = 1.0 - S->b1 - S->b2;
    for (int k = 0; k < 3; ++k) S->N[k] = ld3f(hiN, S->hv[k]);
    S->h = add(add(scl(S->N[0], b0), scl(S->N[1], S->b1)), scl(S->N[2], S->b2));
    S->lh = norm(S->h);
    S->n = scl(S->h, 1.0 / S->lh);
    S->Tf = face_tangent(loV, loF, UV, res, face, &S->c1, &S->c2);
    S->Tt = sub(S->Tf, scl(S->d, dot(S->d, S->Tf)));
    S->lt = norm(S->Tt);
    S->Tp = scl(S->Tt, 1.0 / S->lt);
    S->Bp = scl(cross(S->d, S->Tp), (double)hf);
}

int orc_frozen_forward(const float *loV, int64_t nlv, const int32_t *loF, int64_t nlf, const float *UV,
                       int32_t res, const float *hiV, const int32_t *hiF, const float *hiN, int64_t n,
                       const int32_t *face, const double *bary, const int32_t *g, const int8_t *hf,
                       double *out, double *tb_out) {
    double *s = (double *)malloc(sizeof(double) * (size_t)(3 * (nlv > 0 ? nlv : 1)));
    double *nrm = (double *)malloc(sizeof(double) * (size_t)(3 * (nlv > 0 ? nlv : 1)));
    lo_vertex_sums(loV, nlv, loF, nlf, s);
    for (int64_t v = 0; v < nlv; ++v) st3d(nrm, v, scl(ld3d(s, v), 1.0 / norm(ld3d(s, v))));
    for (int64_t r = 0; r < n; ++r) {
        rstate S;
        ray_forward(loV, loF, nrm, UV, res, hiV, hiF, hiN, face[r], bary + 3 * r, g[r], hf[r], &S);
        st3d(out, r, mk(dot(S.n, S.Tp), dot(S.n, S.Bp), dot(S.n, S.d)));
        if (tb_out) { tb_out[3 * r] = S.t; tb_out[3 * r + 1] = S.b1; tb_out[3 * r + 2] = S.b2; }
    }
    free(nrm);
    free(s);
    return ORC_OK;
}

static v3 vabs(v3 a) { return mk(fabs(a.x), fabs(a.y), fabs(a.z)); }
/* Componentwise bound on |a x b| from |a| and |b|. */
static v3 cross_abs(v3 a, v3 b) {
    return mk(a.y * b.z + a.z * b.y, a.z * b.x + a.x * b.z, a.x * b.y + a.y * b.x);
}
static void acc_abs(double *p, int64_t i, v3 a) {
    if (p) st3d(p, i, add(ld3d(p, i), vabs(a)));
}

/* gloV_abs / ghiN_abs (optional, NULL to skip): per gradient entry, the sum of
 * the magnitudes of the terms that the adjoint adds into it (through the
 * vertex-normal chain, a componentwise bound of the same), the scale to which
 * a floating-point evaluation of the sums is accurate.
 *
 * bnoise / ghiN_sens (optional, NULL to skip): given per ray a bound bnoise[r]
 * on the perturbation of the hit weights beta1, beta2 (so beta0 = 1 - beta1 -
 * beta2 moves by at most twice that), ghiN_sens receives per entry of dL/dhi_N
 * the summed first-order bound of how far its terms beta_k h_bar move:
 *   |d(beta_k h_bar)| <= |d beta_k| |h_bar| + |beta_k| |d h_bar|,
 *   |d h_bar| <= 3 |n_bar| |d h| / |h|^2,  |d h| <= bnoise (|N1 - N0| + |N2 - N0|)
 * (h_bar = (I - n n^T) n_bar / |h|, n = h / |h|: dn = (I - n n^T) dh / |h| and
 * d|h| = n . dh contribute |n_bar| |dh| / |h|^2 twice and once). */
int orc_adjoint(const float *loV, int64_t nlv, const int32_t *loF, int64_t nlf, const float *UV,
                int32_t res, const float *hiV, int64_t nhv, const int32_t *hiF, const float *hiN, int64_t n,
                const int32_t *face, const double *bary, const int32_t *g, const int8_t *hf,
                const double *gout, double *gloV, double *ghiN, double *gloV_abs, double *ghiN_abs,
                const double *bnoise, double *ghiN_sens) {
    double *s = (double *)malloc(sizeof(double) * (size_t)(3 * (nlv > 0 ? nlv : 1)));
    double *nrm = (double *)malloc(sizeof(double) * (size_t)(3 * (nlv > 0 ? nlv : 1)));
    double *nbar = (double *)calloc((size_t)(3 * (nlv > 0 ? nlv : 1)), sizeof(double));
    double *nbar_abs = (double *)calloc((size_t)(3 * (nlv > 0 ? nlv : 1)), sizeof(double));
    lo_vertex_sums(loV, nlv, loF, nlf, s);
    for (int64_t v = 0; v < nlv; ++v) st3d(nrm, v, scl(ld3d(s, v), 1.0 / norm(ld3d(s, v))));
    for (int64_t i = 0; i < 3 * nlv; ++i) gloV[i] = 0;
    for (int64_t i = 0; i < 3 * nhv; ++i) ghiN[i] = 0;
    if (gloV_abs) for (int64_t i = 0; i < 3 * nlv; ++i) gloV_abs[i] = 0;
    if (ghiN_abs) for (int64_t i = 0; i < 3 * nhv; ++i) ghiN_abs[i] = 0;
    if (ghiN_sens) for (int64_t i = 0; i < 3 * nhv; ++i) ghiN_sens[i] = 0;
    for (int64_t r = 0; r < n; ++r) {
        rstate S;
        ray_forward(loV, loF, nrm, UV, res, hiV, hiF, hiN, face[r], bary + 3 * r, g[r], hf[r], &S);
        v3 o = ld3d(gout, r);
        double H = (double)hf[r];
        /* out = (n.T', n.B', n.d), B' = H (d x T') */
        v3 nb = add(add(scl(S.Tp, o.x), scl(S.Bp, o.y)), scl(S.d, o.z));
        v3 Tpb = add(scl(S.n, o.x), scl(cross(S.n, S.d), o.y * H));
        v3 db = add(scl(S.n, o.z), scl(cross(S.Tp, S.n), o.y * H));
        /* T' = T~/|T~| */
        v3 Ttb = scl(sub(Tpb, scl(S.Tp, dot(Tpb, S.Tp))), 1.0 / S.lt);
        /* T~ = T_f - (d.T_f) d */
        v3 Tfb = sub(Ttb, scl(S.d, dot(S.d, Ttb)));
        db = sub(db, add(scl(Ttb, dot(S.d, S.Tf)), scl(S.Tf, dot(S.d, Ttb))));
        /* n = h/|h| */
        v3 hb = scl(sub(nb, scl(S.n, dot(nb, S.n))), 1.0 / S.lh);
        double beta[3] = {1.0 - S.b1 - S.b2, S.b1, S.b2};
        for (int k = 0; k < 3; ++k) {
            st3d(ghiN, S.hv[k], add(ld3d(ghiN, S.hv[k]), scl(hb, beta[k])));
            acc_abs(ghiN_abs, S.hv[k], scl(hb, beta[k]));
        }
        if (ghiN_sens && bnoise) {
            double db = bnoise[r];
            double dh = db * (norm(sub(S.N[1], S.N[0])) + norm(sub(S.N[2], S.N[0])));
            double dhb = 3.0 * norm(nb) * dh / (S.lh * S.lh);
            for (int k = 0; k < 3; ++k) {
                double dbk = k == 0 ? 2.0 * db : db;
                v3 e = add(scl(vabs(hb), dbk), scl(mk(1, 1, 1), fabs(beta[k]) * dhb));
                st3d(ghiN_sens, S.hv[k], add(ld3d(ghiN_sens, S.hv[k]), e));
            }
        }
        double b1b = dot(hb, sub(S.N[1], S.N[0])), b2b = dot(hb, sub(S.N[2], S.N[0]));
        /* [-d | e1 | e2] (t, b1, b2) = p - A: w = M^-T (0, b1b, b2b) */
        v3 md = scl(S.d, -1.0);
        /* M^T w = xbar: rows of M^T are -d, e1, e2 */
        v3 w;
        {
            /* solve M^T w = xb with M^T = [md; e1; e2] (rows) */
            v3 r0 = md, r1 = S.e1, r2 = S.e2;
            /* columns of M^T are (r0.x, r1.x, r2.x) etc.; Cramer on the transposed system */
            v3 c0 = mk(r0.x, r1.x, r2.x), c1 = mk(r0.y, r1.y, r2.y), c2 = mk(r0.z, r1.z, r2.z);
            w = solve3(c0, c1, c2, mk(0.0, b1b, b2b));
        }
        v3 pb = w;
        db = add(db, scl(w, S.t));
        /* d = m/|m| */
        v3 mb = scl(sub(db, scl(S.d, dot(db, S.d))), 1.0 / S.lm);
        const double *bk = bary + 3 * r;
        for (int k = 0; k < 3; ++k) {
            int32_t v = S.lv[k];
            st3d(gloV, v, add(ld3d(gloV, v), scl(pb, bk[k])));
            st3d(nbar, v, add(ld3d(nbar, v), scl(mb, bk[k])));
            acc_abs(gloV_abs, v, scl(pb, bk[k]));
            acc_abs(nbar_abs, v, scl(mb, bk[k]));
        }
        /* T_f = c1 (V1 - V0) + c2 (V2 - V0) */
        v3 e1b = scl(Tfb, S.c1), e2b = scl(Tfb, S.c2);
        st3d(gloV, S.lv[1], add(ld3d(gloV, S.lv[1]), e1b));
        st3d(gloV, S.lv[2], add(ld3d(gloV, S.lv[2]), e2b));
        st3d(gloV, S.lv[0], sub(ld3d(gloV, S.lv[0]), add(e1b, e2b)));
        acc_abs(gloV_abs, S.lv[1], e1b);
        acc_abs(gloV_abs, S.lv[2], e2b);
        acc_abs(gloV_abs, S.lv[0], add(vabs(e1b), vabs(e2b)));
    }
    /* n_v = s_v/|s_v|, s_v = sum of face cross products */
    double *sb = (double *)calloc((size_t)(3 * (nlv > 0 ? nlv : 1)), sizeof(double));
    double *sb_abs = (double *)calloc((size_t)(3 * (nlv > 0 ? nlv : 1)), sizeof(double));
    for (int64_t v = 0; v < nlv; ++v) {
        v3 nv = ld3d(nrm, v), nbv = ld3d(nbar, v);
        double ls = norm(ld3d(s, v));
        st3d(sb, v, scl(sub(nbv, scl(nv, dot(nbv, nv))), 1.0 / ls));
        /* |(I - n n^T) x| <= |x| + |n| (|n| . |x|) componentwise */
        v3 xa = ld3d(nbar_abs, v), na = vabs(nv);
        st3d(sb_abs, v, scl(add(xa, scl(na, dot(na, xa))), 1.0 / ls));
    }
    for (int64_t f = 0; f < nlf; ++f) {
        int32_t a = loF[3 * f], b = loF[3 * f + 1], c = loF[3 * f + 2];
        v3 cb = add(add(ld3d(sb, a), ld3d(sb, b)), ld3d(sb, c));
        v3 A = ld3f(loV, a), B = ld3f(loV, b), C = ld3f(loV, c);
        v3 e1 = sub(B, A), e2 = sub(C, A);
        v3 e1b = cross(e2, cb), e2b = cross(cb, e1);
        st3d(gloV, b, add(ld3d(gloV, b), e1b));
        st3d(gloV, c, add(ld3d(gloV, c), e2b));
        st3d(gloV, a, sub(ld3d(gloV, a), add(e1b, e2b)));
        if (gloV_abs) {
            v3 cba = add(add(ld3d(sb_abs, a), ld3d(sb_abs, b)), ld3d(sb_abs, c));
            v3 e1ba = cross_abs(vabs(e2), cba), e2ba = cross_abs(cba, vabs(e1));
            acc_abs(gloV_abs, b, e1ba);
            acc_abs(gloV_abs, c, e2ba);
            acc_abs(gloV_abs, a, add(e1ba, e2ba));
        }
    }
    free(sb_abs);
    free(nbar_abs);
    free(sb);
    free(nbar);
    free(nrm);
    free(s);
    return ORC_OK;
}
