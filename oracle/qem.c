/*
 * FP64 CPU oracle for quadric-error edge-collapse simplification with the
 * edge-constrained optimal placement of Sec. 6.1 ("Mesh Simplification").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no source, header, table or helper with the GPU
 * library.
 *
 * What the paper fixes:
 *   - every vertex carries a quadric Q_v (4x4, symmetric) whose form
 *     [x;1]^T Q_v [x;1] is the sum of squared distances of x to the planes of
 *     the faces around v;
 *   - collapsing edge (v0, v1) is ranked by min E over the placement, with
 *     Q = Q_v0 + Q_v1;
 *   - interior edges: solve A x = -b (A the upper-left 3x3 block of Q, b its
 *     last column without the corner), project onto the edge with
 *     t = <x - v0, v1 - v0> / |v1 - v0|^2 clamped to [0, 1]; midpoint when the
 *     quadric is singular;
 *   - boundary edges keep boundary vertices fixed or take the endpoint of
 *     lower error;
 *   - the same placement serves the ranking and the collapse.
 *   The original CuMesh placement (midpoint for interior edges) is kept as a
 *   switch, for the comparison the section makes.
 *
 * Readings where the paper is silent (each one a plain rule):
 *   R1 face quadric: c = (p1 - p0) x (p2 - p0), u = (c, -c.p0); K = u u^T / (c.c)
 *      (the unit-normal plane quadric, unweighted); a face with c.c == 0 adds
 *      nothing.  Q_v sums K over the faces around v in ascending face order.
 *   R2 singular: not (det A > 1e-8 (trace A)^3); the solve is the adjugate
 *      over the determinant.  A zero-length edge takes t = 0.
 *   R3 placement p = (1 - t) v0 + t v1 per component (t = 1/2 for the
 *      midpoint).  A vertex is a boundary vertex when one of its edges has a
 *      single face.  Interior edge with one boundary endpoint: p = that
 *      endpoint.  Boundary edge: the endpoint with the lower E (v0 on a tie).
 *   R4 cost = max(E(p), 0) with E written out term by term (below).
 *   R5 an edge (v0 < v1) may collapse only if: it has one or two faces; the
 *      one-rings of v0 and v1 share exactly as many vertices as the edge has
 *      faces (link condition); not both endpoints have exactly three
 *      neighbours (the collapse of a tetrahedron); it is not an interior edge
 *      between two boundary vertices; and every face around v0 or v1 that
 *      does not contain both keeps a normal with positive dot product with its old normal (no fold,
 *      no degenerate face) when its endpoint moves to p.
 *   R6 collapse: v0 (the lower index) survives at p with Q_v0 + Q_v1; faces
 *      that held v1 hold v0; faces that held both disappear (one for a
 *      boundary edge, two for an interior one).
 *
 * Two drivers:
 *   - greedy: the textbook serial order (Garland & Heckbert 1997): always
 *     collapse the cheapest valid edge, until the face count reaches the
 *     target;
 *   - rounds: the parallel schedule (our reading of a parallel collapse; the
 *     paper gives none).  Per round, over the current mesh: edges are numbered
 *     in (v0, v1) order; each valid edge gets the key (float32(cost), id);
 *     the eligible edges are the valid ones whose float32 cost is at most the
 *     k-th smallest, k = ceil(rho n_valid); m(v) = least key of the eligible
 *     edges at v; M(v) = least m over v and its neighbours; an eligible edge
 *     collapses when M(v0) = M(v1) = its key.  No two such edges share a
 *     vertex or a face, nor does one touch the other's one-ring faces, so
 *     they apply in one step.  When they would remove more faces than are
 *     left above the target, the cheapest prefix in key order is kept.  The
 *     rounds end at the target, when nothing collapses, or after max_rounds.
 *   Output: the surviving vertices referenced by a face, in ascending index,
 *   and the surviving faces in ascending index, renumbered.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define QEM_OK 0
#define QEM_EINVAL -1
#define QEM_ENOMEM -2

/* ------------------------------------------------------------------ mesh */

typedef struct {
    int64_t nv, nf;
    double *P;       /* [nv][3] */
    double *Q;       /* [nv][10]: q00 q01 q02 q03 q11 q12 q13 q22 q23 q33 */
    int32_t *F;      /* [nf][3], original face slots */
    uint8_t *falive;
    uint8_t *valive;
    int32_t **fl;    /* faces around each vertex */
    int32_t *fl_n;
    int32_t *fl_cap;
} Mesh;

static int has(const int32_t *f, int32_t v) { return f[0] == v || f[1] == v || f[2] == v; }

static void face_quadric(const double *P, const int32_t *f, double *K) {
    const double *a = P + 3 * (int64_t)f[0], *b = P + 3 * (int64_t)f[1], *c = P + 3 * (int64_t)f[2];
    double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    double cc = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
    double u[4] = {n[0], n[1], n[2], -(n[0] * a[0] + n[1] * a[1] + n[2] * a[2])};
    if (cc == 0) {
        for (int i = 0; i < 10; ++i) K[i] = 0;
        return;
    }
    int k = 0;
    for (int i = 0; i < 4; ++i)
        for (int j = i; j < 4; ++j) K[k++] = (u[i] * u[j]) / cc;
}

/* [x;1]^T Q [x;1], term by term */
static double qerr(const double *q, const double *x) {
    return q[0] * x[0] * x[0] + 2.0 * q[1] * x[0] * x[1] + 2.0 * q[2] * x[0] * x[2] + 2.0 * q[3] * x[0] +
           q[4] * x[1] * x[1] + 2.0 * q[5] * x[1] * x[2] + 2.0 * q[6] * x[1] + q[7] * x[2] * x[2] +
           2.0 * q[8] * x[2] + q[9];
}

static int fl_push(Mesh *m, int32_t v, int32_t f) {
    if (m->fl_n[v] == m->fl_cap[v]) {
        int32_t cap = m->fl_cap[v] ? 2 * m->fl_cap[v] : 8;
        int32_t *p = (int32_t *)realloc(m->fl[v], sizeof(int32_t) * cap);
        if (!p) return QEM_ENOMEM;
        m->fl[v] = p;
        m->fl_cap[v] = cap;
    }
    m->fl[v][m->fl_n[v]++] = f;
    return QEM_OK;
}

static void mesh_free(Mesh *m) {
    if (m->fl)
        for (int64_t v = 0; v < m->nv; ++v) free(m->fl[v]);
    free(m->fl); free(m->fl_n); free(m->fl_cap);
    free(m->P); free(m->Q); free(m->F); free(m->falive); free(m->valive);
    memset(m, 0, sizeof(*m));
}

/* face lists rebuilt from the live faces, each in ascending face order */
static int rebuild_lists(Mesh *m) {
    for (int64_t v = 0; v < m->nv; ++v) m->fl_n[v] = 0;
    for (int64_t f = 0; f < m->nf; ++f) {
        if (!m->falive[f]) continue;
        for (int k = 0; k < 3; ++k)
            if (fl_push(m, m->F[3 * f + k], (int32_t)f)) return QEM_ENOMEM;
    }
    return QEM_OK;
}

/* positions from float (Vf) or double (Vd) input */
static int mesh_init(Mesh *m, const float *Vf, const double *Vd, int64_t nv, const int32_t *F, int64_t nf) {
    memset(m, 0, sizeof(*m));
    m->nv = nv; m->nf = nf;
    m->P = (double *)malloc(sizeof(double) * 3 * (nv ? nv : 1));
    m->Q = (double *)calloc(10 * (nv ? nv : 1), sizeof(double));
    m->F = (int32_t *)malloc(sizeof(int32_t) * 3 * (nf ? nf : 1));
    m->falive = (uint8_t *)malloc(nf ? nf : 1);
    m->valive = (uint8_t *)malloc(nv ? nv : 1);
    m->fl = (int32_t **)calloc(nv ? nv : 1, sizeof(int32_t *));
    m->fl_n = (int32_t *)calloc(nv ? nv : 1, sizeof(int32_t));
    m->fl_cap = (int32_t *)calloc(nv ? nv : 1, sizeof(int32_t));
    if (!m->P || !m->Q || !m->F || !m->falive || !m->valive || !m->fl || !m->fl_n || !m->fl_cap) return QEM_ENOMEM;
    for (int64_t i = 0; i < 3 * nv; ++i) m->P[i] = Vf ? (double)Vf[i] : Vd[i];
    for (int64_t f = 0; f < nf; ++f) {
        for (int k = 0; k < 3; ++k) {
            int32_t v = F[3 * f + k];
            if (v < 0 || v >= nv) return QEM_EINVAL;
            m->F[3 * f + k] = v;
        }
        if (F[3 * f] == F[3 * f + 1] || F[3 * f + 1] == F[3 * f + 2] || F[3 * f] == F[3 * f + 2]) return QEM_EINVAL;
        m->falive[f] = 1;
    }
    for (int64_t v = 0; v < nv; ++v) m->valive[v] = 1;
    int rc = rebuild_lists(m);
    if (rc) return rc;
    /* R1: ascending face order per vertex */
    for (int64_t v = 0; v < nv; ++v) {
        double *q = m->Q + 10 * v;
        for (int32_t i = 0; i < m->fl_n[v]; ++i) {
            double K[10];
            face_quadric(m->P, m->F + 3 * (int64_t)m->fl[v][i], K);
            for (int j = 0; j < 10; ++j) q[j] = q[j] + K[j];
        }
    }
    return QEM_OK;
}

/* unique neighbours of v, ascending; returns the count (buffer grows) */
static int32_t neighbours(const Mesh *m, int32_t v, int32_t **buf, int32_t *cap) {
    int32_t n = 0;
    for (int32_t i = 0; i < m->fl_n[v]; ++i) {
        const int32_t *f = m->F + 3 * (int64_t)m->fl[v][i];
        for (int k = 0; k < 3; ++k) {
            int32_t x = f[k];
            if (x == v) continue;
            int dup = 0;
            for (int32_t j = 0; j < n; ++j)
                if ((*buf)[j] == x) { dup = 1; break; }
            if (dup) continue;
            if (n == *cap) {
                *cap = *cap ? 2 * *cap : 16;
                *buf = (int32_t *)realloc(*buf, sizeof(int32_t) * *cap);
            }
            (*buf)[n++] = x;
        }
    }
    /* insertion sort */
    for (int32_t i = 1; i < n; ++i) {
        int32_t x = (*buf)[i], j = i - 1;
        while (j >= 0 && (*buf)[j] > x) { (*buf)[j + 1] = (*buf)[j]; --j; }
        (*buf)[j + 1] = x;
    }
    return n;
}

/* number of faces around v that also hold w */
static int32_t shared_faces(const Mesh *m, int32_t v, int32_t w) {
    int32_t c = 0;
    for (int32_t i = 0; i < m->fl_n[v]; ++i)
        if (has(m->F + 3 * (int64_t)m->fl[v][i], w)) ++c;
    return c;
}

typedef struct {
    int valid;
    int32_t faces;     /* faces removed by the collapse */
    double cost;
    double p[3];
} EdgeEval;

typedef struct {
    int32_t *a, *b;
    int32_t ca, cb;
} Scratch;

/* does moving vertex `moved` of every face around `moved` that lacks `other`
 * to p keep each face's orientation (R5)? */
static int no_fold(const Mesh *m, int32_t moved, int32_t other, const double *p) {
    for (int32_t i = 0; i < m->fl_n[moved]; ++i) {
        const int32_t *f = m->F + 3 * (int64_t)m->fl[moved][i];
        if (has(f, other)) continue;
        double a[3][3], b[3][3];
        for (int k = 0; k < 3; ++k)
            for (int c = 0; c < 3; ++c) {
                a[k][c] = m->P[3 * (int64_t)f[k] + c];
                b[k][c] = f[k] == moved ? p[c] : a[k][c];
            }
        double e1[3], e2[3], g1[3], g2[3];
        for (int c = 0; c < 3; ++c) {
            e1[c] = a[1][c] - a[0][c]; e2[c] = a[2][c] - a[0][c];
            g1[c] = b[1][c] - b[0][c]; g2[c] = b[2][c] - b[0][c];
        }
        double n0[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        double n1[3] = {g1[1] * g2[2] - g1[2] * g2[1], g1[2] * g2[0] - g1[0] * g2[2], g1[0] * g2[1] - g1[1] * g2[0]};
        double d = n0[0] * n1[0] + n0[1] * n1[1] + n0[2] * n1[2];
        if (!(d > 0)) return 0;
    }
    return 1;
}

/* R2-R5 for edge (v0 < v1) of the current mesh */
static EdgeEval eval_edge(const Mesh *m, int32_t v0, int32_t v1, int midpoint, Scratch *s) {
    EdgeEval e;
    memset(&e, 0, sizeof(e));
    int32_t c = shared_faces(m, v0, v1);
    e.faces = c;
    if (c < 1 || c > 2) return e;
    int32_t na = neighbours(m, v0, &s->a, &s->ca);
    int32_t nb = neighbours(m, v1, &s->b, &s->cb);
    int32_t common = 0;
    for (int32_t i = 0; i < na; ++i)
        for (int32_t j = 0; j < nb; ++j)
            if (s->a[i] == s->b[j]) ++common;
    if (common != c) return e;
    if (na == 3 && nb == 3) return e;
    int b0 = 0, b1 = 0;
    for (int32_t i = 0; i < na; ++i)
        if (shared_faces(m, v0, s->a[i]) == 1) { b0 = 1; break; }
    for (int32_t j = 0; j < nb; ++j)
        if (shared_faces(m, v1, s->b[j]) == 1) { b1 = 1; break; }
    int bedge = c == 1;
    if (!bedge && b0 && b1) return e;

    double q[10];
    const double *q0 = m->Q + 10 * (int64_t)v0, *q1 = m->Q + 10 * (int64_t)v1;
    for (int i = 0; i < 10; ++i) q[i] = q0[i] + q1[i];
    const double *p0 = m->P + 3 * (int64_t)v0, *p1 = m->P + 3 * (int64_t)v1;
    double p[3];
    if (bedge) {
        double e0 = qerr(q, p0), e1 = qerr(q, p1);
        const double *src = e1 < e0 ? p1 : p0;
        p[0] = src[0]; p[1] = src[1]; p[2] = src[2];
    } else if (b0) {
        p[0] = p0[0]; p[1] = p0[1]; p[2] = p0[2];
    } else if (b1) {
        p[0] = p1[0]; p[1] = p1[1]; p[2] = p1[2];
    } else {
        double t = 0.5;
        if (!midpoint) {
            double det = q[0] * (q[4] * q[7] - q[5] * q[5]) - q[1] * (q[1] * q[7] - q[5] * q[2]) +
                         q[2] * (q[1] * q[5] - q[4] * q[2]);
            double tr = q[0] + q[4] + q[7];
            if (det > 1e-8 * tr * tr * tr) {
                double i00 = q[4] * q[7] - q[5] * q[5], i01 = q[2] * q[5] - q[1] * q[7];
                double i02 = q[1] * q[5] - q[2] * q[4], i11 = q[0] * q[7] - q[2] * q[2];
                double i12 = q[1] * q[2] - q[0] * q[5], i22 = q[0] * q[4] - q[1] * q[1];
                double x[3];
                x[0] = -(i00 * q[3] + i01 * q[6] + i02 * q[8]) / det;
                x[1] = -(i01 * q[3] + i11 * q[6] + i12 * q[8]) / det;
                x[2] = -(i02 * q[3] + i12 * q[6] + i22 * q[8]) / det;
                double d[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
                double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (dd > 0) {
                    t = ((x[0] - p0[0]) * d[0] + (x[1] - p0[1]) * d[1] + (x[2] - p0[2]) * d[2]) / dd;
                    if (!(t > 0)) t = 0;
                    if (t > 1) t = 1;
                } else {
                    t = 0;
                }
            }
        }
        for (int k = 0; k < 3; ++k) p[k] = (1.0 - t) * p0[k] + t * p1[k];
    }
    double E = qerr(q, p);
    if (!(E == E)) return e;
    e.cost = E > 0 ? E : 0;
    e.p[0] = p[0]; e.p[1] = p[1]; e.p[2] = p[2];
    if (!no_fold(m, v0, v1, p) || !no_fold(m, v1, v0, p)) return e;
    e.valid = 1;
    return e;
}

/* R6 */
static int collapse(Mesh *m, int32_t v0, int32_t v1, const double *p) {
    m->P[3 * (int64_t)v0] = p[0]; m->P[3 * (int64_t)v0 + 1] = p[1]; m->P[3 * (int64_t)v0 + 2] = p[2];
    double *q0 = m->Q + 10 * (int64_t)v0;
    const double *q1 = m->Q + 10 * (int64_t)v1;
    for (int i = 0; i < 10; ++i) q0[i] = q0[i] + q1[i];
    m->valive[v1] = 0;
    int removed = 0;
    for (int32_t i = 0; i < m->fl_n[v1]; ++i) {
        int32_t f = m->fl[v1][i];
        int32_t *fv = m->F + 3 * (int64_t)f;
        if (has(fv, v0)) {
            m->falive[f] = 0;
            ++removed;
        } else {
            for (int k = 0; k < 3; ++k)
                if (fv[k] == v1) fv[k] = v0;
            if (fl_push(m, v0, f)) return -1;
        }
    }
    m->fl_n[v1] = 0;
    /* drop dead faces from the survivor's list (and from the lists of the
     * removed faces' third vertices) */
    int32_t k = 0;
    for (int32_t i = 0; i < m->fl_n[v0]; ++i)
        if (m->falive[m->fl[v0][i]]) m->fl[v0][k++] = m->fl[v0][i];
    m->fl_n[v0] = k;
    return removed;
}

static void drop_dead(Mesh *m, int32_t v) {
    int32_t k = 0;
    for (int32_t i = 0; i < m->fl_n[v]; ++i)
        if (m->falive[m->fl[v][i]]) m->fl[v][k++] = m->fl[v][i];
    m->fl_n[v] = k;
}

static int emit(const Mesh *m, double *V_out, int32_t *F_out, int64_t *counts) {
    int32_t *map = (int32_t *)malloc(sizeof(int32_t) * (m->nv ? m->nv : 1));
    if (!map) return QEM_ENOMEM;
    for (int64_t v = 0; v < m->nv; ++v) map[v] = -1;
    for (int64_t f = 0; f < m->nf; ++f)
        if (m->falive[f])
            for (int k = 0; k < 3; ++k) map[m->F[3 * f + k]] = 0;
    int64_t nv = 0, nf = 0;
    for (int64_t v = 0; v < m->nv; ++v)
        if (map[v] == 0) {
            map[v] = (int32_t)nv;
            for (int c = 0; c < 3; ++c) V_out[3 * nv + c] = m->P[3 * v + c];
            ++nv;
        }
    for (int64_t f = 0; f < m->nf; ++f)
        if (m->falive[f]) {
            for (int k = 0; k < 3; ++k) F_out[3 * nf + k] = map[m->F[3 * f + k]];
            ++nf;
        }
    counts[0] = nv;
    counts[1] = nf;
    free(map);
    return QEM_OK;
}

static uint32_t f32_bits(double c) {
    float f = (float)c;
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

/* ------------------------------------------------------------ entry points */

/* Per-vertex quadrics of the input mesh (R1): Q_out [nv][10]. */
int orc_qem_quadrics(const float *V, int64_t nv, const int32_t *F, int64_t nf, double *Q_out) {
    Mesh m;
    int rc = mesh_init(&m, V, NULL, nv, F, nf);
    if (rc == QEM_OK) memcpy(Q_out, m.Q, sizeof(double) * 10 * nv);
    mesh_free(&m);
    return rc;
}

/* Every edge of a mesh in (v0, v1) order with its collapse (R2-R5): FP64
 * positions V, and the vertex quadrics Q [nv][10] (NULL: from the faces, R1);
 * edges_out [cap][2], valid_out, faces_out, cost_out, p_out [cap][3];
 * *n_edges = count (QEM_EINVAL when it exceeds cap). */
int orc_qem_edges(const double *V, int64_t nv, const int32_t *F, int64_t nf, const double *Q, int32_t midpoint,
                  int64_t cap, int32_t *edges_out, uint8_t *valid_out, int32_t *faces_out, double *cost_out,
                  double *p_out, int64_t *n_edges) {
    Mesh m;
    Scratch s = {0};
    int32_t *nb = NULL, ncap = 0;
    int rc = mesh_init(&m, NULL, V, nv, F, nf);
    if (rc == QEM_OK && Q) memcpy(m.Q, Q, sizeof(double) * 10 * nv);
    int64_t ne = 0;
    for (int64_t v = 0; rc == QEM_OK && v < nv; ++v) {
        int32_t n = neighbours(&m, (int32_t)v, &nb, &ncap);
        for (int32_t i = 0; i < n; ++i) {
            int32_t w = nb[i];
            if (w <= v) continue;
            if (ne >= cap) { rc = QEM_EINVAL; break; }
            EdgeEval e = eval_edge(&m, (int32_t)v, w, midpoint, &s);
            edges_out[2 * ne] = (int32_t)v; edges_out[2 * ne + 1] = w;
            valid_out[ne] = (uint8_t)e.valid; faces_out[ne] = e.faces; cost_out[ne] = e.cost;
            for (int c = 0; c < 3; ++c) p_out[3 * ne + c] = e.p[c];
            ++ne;
        }
    }
    *n_edges = ne;
    free(nb); free(s.a); free(s.b);
    mesh_free(&m);
    return rc;
}

typedef struct {
    uint64_t key;
    int64_t id;
} KeyId;

static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : x > y;
}

static int cmp_key(const void *a, const void *b) {
    uint64_t x = ((const KeyId *)a)->key, y = ((const KeyId *)b)->key;
    return x < y ? -1 : x > y;
}

/* The round schedule.  stats_out (optional) [max_rounds][4]: edges, valid
 * edges, collapses, faces after the round; *rounds_out = rounds run. */
int orc_qem_rounds(const float *V, int64_t nv, const int32_t *F, int64_t nf, int64_t target, double rho,
                   int32_t max_rounds, int32_t midpoint, double *V_out, int32_t *F_out, int64_t *counts,
                   int64_t *stats_out, int32_t *rounds_out) {
    if (target < 4 || !(rho > 0 && rho <= 1) || max_rounds < 0) return QEM_EINVAL;
    Mesh m;
    int rc = mesh_init(&m, V, NULL, nv, F, nf);
    Scratch s = {0};
    int32_t *nb = NULL, ncap = 0;
    int64_t ecap = 0;
    int32_t *E = NULL;
    EdgeEval *ev = NULL;
    uint64_t *key = NULL, *mv = NULL, *Mv = NULL;
    uint32_t *bits = NULL;
    KeyId *win = NULL;
    int64_t live = nf;
    int32_t round = 0;
    while (rc == QEM_OK && live > target && round < max_rounds) {
        rc = rebuild_lists(&m);
        if (rc) break;
        /* edges in (v0, v1) order */
        int64_t ne = 0;
        for (int64_t v = 0; v < nv; ++v) {
            int32_t n = neighbours(&m, (int32_t)v, &nb, &ncap);
            for (int32_t i = 0; i < n; ++i) {
                if (nb[i] <= v) continue;
                if (ne == ecap) {
                    ecap = ecap ? 2 * ecap : 1024;
                    E = (int32_t *)realloc(E, sizeof(int32_t) * 2 * ecap);
                    ev = (EdgeEval *)realloc(ev, sizeof(EdgeEval) * ecap);
                    key = (uint64_t *)realloc(key, sizeof(uint64_t) * ecap);
                    bits = (uint32_t *)realloc(bits, sizeof(uint32_t) * ecap);
                    win = (KeyId *)realloc(win, sizeof(KeyId) * ecap);
                    if (!E || !ev || !key || !bits || !win) { rc = QEM_ENOMEM; break; }
                }
                E[2 * ne] = (int32_t)v; E[2 * ne + 1] = nb[i];
                ++ne;
            }
            if (rc) break;
        }
        if (rc) break;
        int64_t nvalid = 0;
        for (int64_t e = 0; e < ne; ++e) {
            ev[e] = eval_edge(&m, E[2 * e], E[2 * e + 1], midpoint, &s);
            key[e] = ((uint64_t)f32_bits(ev[e].cost) << 32) | (uint64_t)(uint32_t)e;
            if (ev[e].valid) bits[nvalid++] = f32_bits(ev[e].cost);
        }
        int64_t nwin = 0, removed = 0;
        if (nvalid > 0) {
            int64_t k = (int64_t)ceil(rho * (double)nvalid);
            if (k < 1) k = 1;
            if (k > nvalid) k = nvalid;
            qsort(bits, nvalid, sizeof(uint32_t), cmp_u32);
            uint32_t tau = bits[k - 1];
            if (!mv) {
                mv = (uint64_t *)malloc(sizeof(uint64_t) * nv);
                Mv = (uint64_t *)malloc(sizeof(uint64_t) * nv);
                if (!mv || !Mv) { rc = QEM_ENOMEM; break; }
            }
            for (int64_t v = 0; v < nv; ++v) mv[v] = UINT64_MAX;
            for (int64_t e = 0; e < ne; ++e) {
                if (!ev[e].valid || (uint32_t)(key[e] >> 32) > tau) continue;
                int32_t a = E[2 * e], b = E[2 * e + 1];
                if (key[e] < mv[a]) mv[a] = key[e];
                if (key[e] < mv[b]) mv[b] = key[e];
            }
            for (int64_t v = 0; v < nv; ++v) Mv[v] = mv[v];
            for (int64_t e = 0; e < ne; ++e) {
                int32_t a = E[2 * e], b = E[2 * e + 1];
                if (mv[b] < Mv[a]) Mv[a] = mv[b];
                if (mv[a] < Mv[b]) Mv[b] = mv[a];
            }
            int64_t total = 0;
            for (int64_t e = 0; e < ne; ++e) {
                if (!ev[e].valid || (uint32_t)(key[e] >> 32) > tau) continue;
                if (Mv[E[2 * e]] == key[e] && Mv[E[2 * e + 1]] == key[e]) {
                    win[nwin].key = key[e];
                    win[nwin].id = e;
                    total += ev[e].faces;
                    ++nwin;
                }
            }
            int64_t budget = live - target;
            if (total > budget) {
                qsort(win, nwin, sizeof(KeyId), cmp_key);
                int64_t cum = 0, keep = 0;
                while (keep < nwin && cum + ev[win[keep].id].faces <= budget) cum += ev[win[keep++].id].faces;
                nwin = keep;
            }
            for (int64_t i = 0; i < nwin; ++i) {
                int64_t e = win[i].id;
                int r = collapse(&m, E[2 * e], E[2 * e + 1], ev[e].p);
                if (r < 0) { rc = QEM_ENOMEM; break; }
                removed += r;
            }
        }
        live -= removed;
        if (stats_out) {
            stats_out[4 * round] = ne; stats_out[4 * round + 1] = nvalid;
            stats_out[4 * round + 2] = nwin; stats_out[4 * round + 3] = live;
        }
        ++round;
        if (nwin == 0) break;
    }
    if (rc == QEM_OK) rc = emit(&m, V_out, F_out, counts);
    if (rounds_out) *rounds_out = round;
    free(E); free(ev); free(key); free(bits); free(win); free(mv); free(Mv);
    free(nb); free(s.a); free(s.b);
    mesh_free(&m);
    return rc;
}

/* ---------------------------------------------------------------- greedy */

typedef struct {
    double cost;
    int32_t v0, v1;
    uint32_t s0, s1;   /* vertex stamps when evaluated */
} HeapItem;

typedef struct {
    HeapItem *a;
    int64_t n, cap;
} Heap;

static int item_less(const HeapItem *x, const HeapItem *y) {
    if (x->cost != y->cost) return x->cost < y->cost;
    if (x->v0 != y->v0) return x->v0 < y->v0;
    return x->v1 < y->v1;
}

static int heap_push(Heap *h, HeapItem it) {
    if (h->n == h->cap) {
        h->cap = h->cap ? 2 * h->cap : 1024;
        h->a = (HeapItem *)realloc(h->a, sizeof(HeapItem) * h->cap);
        if (!h->a) return QEM_ENOMEM;
    }
    int64_t i = h->n++;
    h->a[i] = it;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!item_less(&h->a[i], &h->a[p])) break;
        HeapItem t = h->a[i]; h->a[i] = h->a[p]; h->a[p] = t;
        i = p;
    }
    return QEM_OK;
}

static HeapItem heap_pop(Heap *h) {
    HeapItem top = h->a[0];
    h->a[0] = h->a[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < h->n && item_less(&h->a[l], &h->a[s])) s = l;
        if (r < h->n && item_less(&h->a[r], &h->a[s])) s = r;
        if (s == i) break;
        HeapItem t = h->a[i]; h->a[i] = h->a[s]; h->a[s] = t;
        i = s;
    }
    return top;
}

/* push every valid edge at v with the current stamps */
static int push_edges_at(Mesh *m, int32_t v, int midpoint, const uint32_t *stamp, Heap *h, Scratch *s,
                         int32_t **nb, int32_t *ncap) {
    int32_t n = neighbours(m, v, nb, ncap);
    for (int32_t i = 0; i < n; ++i) {
        int32_t w = (*nb)[i];
        int32_t a = v < w ? v : w, b = v < w ? w : v;
        EdgeEval e = eval_edge(m, a, b, midpoint, s);
        if (!e.valid) continue;
        HeapItem it = {e.cost, a, b, stamp[a], stamp[b]};
        if (heap_push(h, it)) return QEM_ENOMEM;
    }
    return QEM_OK;
}

/* The serial greedy order: *collapses_out = collapses made. */
int orc_qem_greedy(const float *V, int64_t nv, const int32_t *F, int64_t nf, int64_t target, int32_t midpoint,
                   double *V_out, int32_t *F_out, int64_t *counts, int64_t *collapses_out) {
    if (target < 4) return QEM_EINVAL;
    Mesh m;
    int rc = mesh_init(&m, V, NULL, nv, F, nf);
    Scratch s = {0};
    int32_t *nb = NULL, ncap = 0, *ring = NULL, rcap = 0;
    Heap h = {0};
    uint32_t *stamp = (uint32_t *)calloc(nv ? nv : 1, sizeof(uint32_t));
    if (!stamp) rc = QEM_ENOMEM;
    /* every edge once, from its lower endpoint */
    for (int64_t v = 0; rc == QEM_OK && v < nv; ++v) {
        int32_t n = neighbours(&m, (int32_t)v, &nb, &ncap);
        for (int32_t i = 0; i < n; ++i) {
            if (nb[i] <= v) continue;
            EdgeEval e = eval_edge(&m, (int32_t)v, nb[i], midpoint, &s);
            if (!e.valid) continue;
            HeapItem it = {e.cost, (int32_t)v, nb[i], 0, 0};
            if (heap_push(&h, it)) { rc = QEM_ENOMEM; break; }
        }
    }
    int64_t live = nf, done = 0;
    while (rc == QEM_OK && live > target && h.n > 0) {
        HeapItem it = heap_pop(&h);
        if (!m.valive[it.v0] || !m.valive[it.v1]) continue;
        if (it.s0 != stamp[it.v0] || it.s1 != stamp[it.v1]) continue;
        EdgeEval e = eval_edge(&m, it.v0, it.v1, midpoint, &s);
        if (!e.valid) continue;
        if (e.faces > live - target) continue;
        int r = collapse(&m, it.v0, it.v1, e.p);
        if (r < 0) { rc = QEM_ENOMEM; break; }
        live -= r;
        ++done;
        /* the faces around the survivor changed: clean the lists of its
         * neighbours, bump the stamps of the survivor and its ring, and
         * re-evaluate every edge that touches them */
        int32_t n = neighbours(&m, it.v0, &ring, &rcap);
        drop_dead(&m, it.v0);
        for (int32_t i = 0; i < n; ++i) drop_dead(&m, ring[i]);
        stamp[it.v0]++;
        for (int32_t i = 0; i < n; ++i) stamp[ring[i]]++;
        rc = push_edges_at(&m, it.v0, midpoint, stamp, &h, &s, &nb, &ncap);
        for (int32_t i = 0; rc == QEM_OK && i < n; ++i)
            rc = push_edges_at(&m, ring[i], midpoint, stamp, &h, &s, &nb, &ncap);
    }
    if (rc == QEM_OK) rc = emit(&m, V_out, F_out, counts);
    if (collapses_out) *collapses_out = done;
    free(h.a); free(stamp); free(nb); free(ring); free(s.a); free(s.b);
    mesh_free(&m);
    return rc;
}
