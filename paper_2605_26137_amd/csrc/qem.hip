// Quadric-error edge-collapse simplification with the edge-constrained optimal
// placement (Sec. 6.1, after Garland & Heckbert 1997), as parallel rounds.
//
// What the section fixes: a quadric Q_v per vertex (squared distances to the
// planes of its faces), the merged quadric Q = Q_v0 + Q_v1 of an edge, the
// placement (solve A x = -b, project onto the edge with t clamped to [0, 1],
// midpoint when A is singular; boundary vertices stay, a boundary edge takes
// its endpoint of lower error), and the same placement for ranking and
// collapse.  The rest are plain rules of this implementation:
//   face quadric      u = (c, -c.p0) with c = (p1 - p0) x (p2 - p0),
//                     K = u u^T / (c.c), nothing for c.c = 0; Q_v sums K over
//                     the faces of v in ascending face order;
//   singular          not (det A > 1e-8 (trace A)^3); solve by the adjugate;
//   cost              max(E(p), 0), E written term by term;
//   valid collapse    one or two faces on the edge, link condition (the rings
//                     share exactly that many vertices), not two endpoints of
//                     three neighbours each (a tetrahedron), not an interior
//                     edge between boundary vertices, and no face around an
//                     endpoint turned to a non-positive dot with its old
//                     normal by the move;
//   a round           edges numbered in (v0, v1) order get the key
//                     (float32(cost) bits, id); eligible = valid with float32
//                     cost <= the k-th smallest, k = ceil(rho n_valid);
//                     m(v) = least eligible key at v, M(v) = least m over v and
//                     its ring; an eligible edge with M(v0) = M(v1) = its key
//                     collapses (no two such edges touch each other's faces);
//                     when they would remove more faces than are left above
//                     the target, only the prefix in key order that fits;
//   collapse          v0 (lower index) survives at p with Q_v0 + Q_v1, faces
//                     holding both endpoints disappear, the others keep their
//                     order.
// All quadric, placement, cost and orientation arithmetic is FP64 with no
// contraction, so every discrete decision (validity, order, singularity)
// follows the plain definition above on the exact FP64 values.
//
// Layout (all in the caller's workspace): positions P [nv][3] and quadrics
// Q [nv][10] in FP64 (q00 q01 q02 q03 q11 q12 q13 q22 q23 q33); the live faces
// [live][3] compacted in their original order after every round; per round
// the vertex -> face lists (CSR), the sorted unique neighbour lists (CSR), the
// edges [ne][2], their float32 cost bits (0xFFFFFFFF: not collapsible), face
// counts and FP64 placements, and the winner keys.
#pragma clang fp contract(off)

#include <algorithm>
#include <utility>

#include "internal.h"

namespace bake {

namespace {

constexpr int kQB = 256;                    // threads per block of the per-element kernels
constexpr uint32_t kNoKey = 0xFFFFFFFFu;    // cost bits of a non-collapsible edge
constexpr int kSortCap = 32;                // neighbours sorted in LDS per vertex (more: direct ranking)

inline int64_t blocks_for(int64_t n) { return n <= 0 ? 1 : (n + kQB - 1) / kQB; }


__device__ __forceinline__ bool holds(const int32_t* f, int32_t x) { return f[0] == x || f[1] == x || f[2] == x; }

__device__ __forceinline__ uint32_t f32_bits(double c) { return __float_as_uint((float)c); }

// [x;1]^T Q [x;1]
__device__ __forceinline__ double qerr(const double* q, const double* x) {
    return q[0] * x[0] * x[0] + 2.0 * q[1] * x[0] * x[1] + 2.0 * q[2] * x[0] * x[2] + 2.0 * q[3] * x[0] +
           q[4] * x[1] * x[1] + 2.0 * q[5] * x[1] * x[2] + 2.0 * q[6] * x[1] + q[7] * x[2] * x[2] +
           2.0 * q[8] * x[2] + q[9];
}

// ---- set-up -------------------------------------------------------------

__global__ void qem_init_kernel(const float* __restrict__ V, int64_t nv, const int32_t* __restrict__ Fin,
                                int64_t nf, double* __restrict__ P, int32_t* __restrict__ partner,
                                int32_t* __restrict__ F, uint32_t* __restrict__ status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nv) {
        P[3 * i] = (double)V[3 * i];
        P[3 * i + 1] = (double)V[3 * i + 1];
        P[3 * i + 2] = (double)V[3 * i + 2];
        partner[i] = -1;
    }
    if (i < nf) {
        int32_t a = Fin[3 * i], b = Fin[3 * i + 1], c = Fin[3 * i + 2];
        bool bad = a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv || a == b || b == c || a == c;
        if (bad) {
            atomicOr(status, 1u);
            a = b = c = 0;  // keep later passes in bounds; the call fails after set-up
        }
        F[3 * i] = a;
        F[3 * i + 1] = b;
        F[3 * i + 2] = c;
    }
}

// ---- vertex -> face lists -------------------------------------------------

// A face with a repeated vertex (only the stand-in for a bad input face, which
// fails the call after set-up) joins no vertex's list: every list then holds
// distinct faces.
__device__ __forceinline__ bool proper(const int32_t* f) { return f[0] != f[1] && f[1] != f[2] && f[0] != f[2]; }

__global__ void qem_deg_kernel(const int32_t* __restrict__ F, int64_t live, uint32_t* __restrict__ deg) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= live || !proper(F + 3 * f)) return;
    for (int k = 0; k < 3; ++k) atomicAdd(&deg[F[3 * f + k]], 1u);
}

__global__ void qem_adj_kernel(const int32_t* __restrict__ F, int64_t live, const uint32_t* __restrict__ off,
                               uint32_t* __restrict__ cur, uint32_t* __restrict__ adj) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= live || !proper(F + 3 * f)) return;
    for (int k = 0; k < 3; ++k) {
        const int32_t v = F[3 * f + k];
        const uint32_t slot = atomicAdd(&cur[v], 1u);
        adj[off[v] + slot] = (uint32_t)f;
    }
}

// Q_v = sum of the face quadrics around v in ascending face order (the
// unordered list is walked by repeated minimum search).
__global__ void qem_quadric_kernel(const double* __restrict__ P, const int32_t* __restrict__ F, int64_t nv,
                                   const uint32_t* __restrict__ off, const uint32_t* __restrict__ adj,
                                   double* __restrict__ Q) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const uint32_t b = off[v], n = off[v + 1] - b;
    double q[10];
    for (int j = 0; j < 10; ++j) q[j] = 0.0;
    int64_t last = -1;
    for (uint32_t it = 0; it < n; ++it) {
        int64_t f = INT64_MAX;
        for (uint32_t i = 0; i < n; ++i) {
            const int64_t g = adj[b + i];
            if (g > last && g < f) f = g;
        }
        if (f == INT64_MAX) break;  // (the list's faces are distinct: not reached)
        last = f;
        const int32_t* fv = F + 3 * f;
        const double* a = P + 3 * (int64_t)fv[0];
        const double* pb = P + 3 * (int64_t)fv[1];
        const double* pc = P + 3 * (int64_t)fv[2];
        const double e1[3] = {pb[0] - a[0], pb[1] - a[1], pb[2] - a[2]};
        const double e2[3] = {pc[0] - a[0], pc[1] - a[1], pc[2] - a[2]};
        const double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                             e1[0] * e2[1] - e1[1] * e2[0]};
        const double cc = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        if (cc == 0.0) continue;
        const double u[4] = {c[0], c[1], c[2], -(c[0] * a[0] + c[1] * a[1] + c[2] * a[2])};
        int k = 0;
        for (int i = 0; i < 4; ++i)
            for (int j = i; j < 4; ++j) {
                q[k] = q[k] + (u[i] * u[j]) / cc;
                ++k;
            }
    }
    for (int j = 0; j < 10; ++j) Q[10 * v + j] = q[j];
}

// ---- unique neighbours ----------------------------------------------------

// Is vertex x (taken from the i-th face of v's list) seen in an earlier face?
__device__ __forceinline__ bool seen_before(const int32_t* F, const uint32_t* adj, uint32_t b, uint32_t i,
                                            int32_t x) {
    for (uint32_t j = 0; j < i; ++j)
        if (holds(F + 3 * (int64_t)adj[b + j], x)) return true;
    return false;
}

__device__ __forceinline__ uint32_t shared_count(const int32_t* F, const uint32_t* adj, uint32_t b, uint32_t n,
                                                 int32_t x) {
    uint32_t c = 0;
    for (uint32_t j = 0; j < n; ++j) c += holds(F + 3 * (int64_t)adj[b + j], x) ? 1u : 0u;
    return c;
}

// The rings.  Around v, the other two corners of every face name v's
// neighbours, each once per face it shares with v: sorted, the runs of that
// list are the unique neighbours in ascending order, and a run of length one
// is an edge with a single face (v is then a boundary vertex).  The list is
// gathered and insertion-sorted in LDS; vertices with more than kRingFaces
// faces take a slower path over global memory.
// A ring entry is (x << 3) | min(faces shared with x, 7): the ring carries
// each edge's face count for the per-edge evaluation (vertex indices are
// below 2^28).
//   count pass: unique neighbours, neighbours above v, boundary flag, and
//               rings of up to kRingKeep vertices kept at keep[v][...];
//   write pass: the sorted ring into nbr[noff[v] ...] and the edges (v, x),
//               x > v ascending, from eoff[v] (from keep when it holds the
//               ring, else gathered again).
constexpr int kRB = 128;        // threads per block of the ring kernels
constexpr int kRingFaces = 24;  // faces per vertex sorted in LDS
constexpr int kRingKeep = 16;   // ring entries kept per vertex between the two passes

template <bool WRITE>
__global__ void __launch_bounds__(kRB) qem_ring_kernel(const int32_t* __restrict__ F, int64_t nv,
                                                       const uint32_t* __restrict__ off,
                                                       const uint32_t* __restrict__ adj, uint32_t* __restrict__ ncnt,
                                                       uint32_t* __restrict__ hcnt, uint32_t* __restrict__ bnd,
                                                       const uint32_t* __restrict__ noff,
                                                       const uint32_t* __restrict__ eoff, int32_t* __restrict__ nbr,
                                                       int32_t* __restrict__ E, int32_t* __restrict__ keep) {
    __shared__ int32_t ent[2 * kRingFaces][kRB];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const uint32_t b = off[v], n = off[v + 1] - b;
    const int t = threadIdx.x;
    if (WRITE && n <= (uint32_t)kRingFaces && ncnt[v] <= (uint32_t)kRingKeep) {
        const uint32_t m = ncnt[v];
        const int32_t* kv = keep + (int64_t)kRingKeep * v;
        uint32_t e = eoff[v], r = noff[v];
        for (uint32_t j = 0; j < m; ++j) {
            const int32_t code = kv[j], x = code >> 3;
            nbr[r++] = code;
            if (x > (int32_t)v) {
                E[2 * (int64_t)e] = (int32_t)v;
                E[2 * (int64_t)e + 1] = x;
                ++e;
            }
        }
        return;
    }
    if (n <= (uint32_t)kRingFaces) {
        uint32_t m = 0;
        for (uint32_t i = 0; i < n; ++i) {
            const int32_t* f = F + 3 * (int64_t)adj[b + i];
            const int32_t c0 = f[0], c1 = f[1], c2 = f[2];
            const int32_t x = c0 == (int32_t)v ? c1 : c0;
            const int32_t y = c2 == (int32_t)v ? c1 : c2;
            // insertion of x, then y, into the sorted prefix
            uint32_t j = m;
            while (j > 0 && ent[j - 1][t] > x) {
                ent[j][t] = ent[j - 1][t];
                --j;
            }
            ent[j][t] = x;
            ++m;
            j = m;
            while (j > 0 && ent[j - 1][t] > y) {
                ent[j][t] = ent[j - 1][t];
                --j;
            }
            ent[j][t] = y;
            ++m;
        }
        uint32_t uniq = 0, higher = 0, boundary = 0;
        uint32_t e = WRITE ? eoff[v] : 0, r = WRITE ? noff[v] : 0;
        for (uint32_t i = 0; i < m;) {
            const int32_t x = ent[i][t];
            uint32_t k = i + 1;
            while (k < m && ent[k][t] == x) ++k;
            if (k - i == 1) boundary = 1;
            const int32_t code = (x << 3) | (int32_t)(k - i < 7 ? k - i : 7);
            if (!WRITE && uniq < (uint32_t)kRingKeep) keep[(int64_t)kRingKeep * v + uniq] = code;
            ++uniq;
            if (WRITE) {
                nbr[r++] = code;
                if (x > (int32_t)v) {
                    E[2 * (int64_t)e] = (int32_t)v;
                    E[2 * (int64_t)e + 1] = x;
                    ++e;
                }
            } else if (x > (int32_t)v) {
                ++higher;
            }
            i = k;
        }
        if (!WRITE) {
            ncnt[v] = uniq;
            hcnt[v] = higher;
            bnd[v] = boundary;
        }
        return;
    }
    // many faces: the same quantities straight from the face list
    uint32_t uniq = 0, higher = 0, boundary = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const int32_t* f = F + 3 * (int64_t)adj[b + i];
        for (int k = 0; k < 3; ++k) {
            const int32_t x = f[k];
            if (x == (int32_t)v || seen_before(F, adj, b, i, x)) continue;
            if (!WRITE) {
                ++uniq;
                if (x > (int32_t)v) ++higher;
                if (shared_count(F, adj, b, n, x) == 1) boundary = 1;
                continue;
            }
            uint32_t below = 0, below_hi = 0;
            for (uint32_t i2 = 0; i2 < n; ++i2) {
                const int32_t* g = F + 3 * (int64_t)adj[b + i2];
                for (int k2 = 0; k2 < 3; ++k2) {
                    const int32_t y = g[k2];
                    if (y == (int32_t)v || y >= x || seen_before(F, adj, b, i2, y)) continue;
                    ++below;
                    if (y > (int32_t)v) ++below_hi;
                }
            }
            const uint32_t sc = shared_count(F, adj, b, n, x);
            nbr[noff[v] + below] = (x << 3) | (int32_t)(sc < 7 ? sc : 7);
            if (x > (int32_t)v) {
                const int64_t e = (int64_t)eoff[v] + below_hi;
                E[2 * e] = (int32_t)v;
                E[2 * e + 1] = x;
            }
        }
    }
    if (!WRITE) {
        ncnt[v] = uniq;
        hcnt[v] = higher;
        bnd[v] = boundary;
    }
}

// ---- per-edge collapse ----------------------------------------------------

// Faces around `moved` that lack `other` keep a positive dot of old and new
// normal when `moved` (now at pm) goes to p; only the other two corners are
// loaded.
__device__ bool no_fold(const double* P, const int32_t* F, const uint32_t* adj, uint32_t b, uint32_t n,
                        int32_t moved, int32_t other, const double* pm, const double* p) {
    for (uint32_t i = 0; i < n; ++i) {
        const int32_t* f = F + 3 * (int64_t)adj[b + i];
        const int32_t f0 = f[0], f1 = f[1], f2 = f[2];
        if (f0 == other || f1 == other || f2 == other) continue;
        const int32_t fk[3] = {f0, f1, f2};
        double a[3][3], q[3][3];
        for (int k = 0; k < 3; ++k) {
            if (fk[k] == moved) {
                for (int c = 0; c < 3; ++c) {
                    a[k][c] = pm[c];
                    q[k][c] = p[c];
                }
            } else {
                const double* src = P + 3 * (int64_t)fk[k];
                for (int c = 0; c < 3; ++c) {
                    a[k][c] = src[c];
                    q[k][c] = src[c];
                }
            }
        }
        double e1[3], e2[3], g1[3], g2[3];
        for (int c = 0; c < 3; ++c) {
            e1[c] = a[1][c] - a[0][c];
            e2[c] = a[2][c] - a[0][c];
            g1[c] = q[1][c] - q[0][c];
            g2[c] = q[2][c] - q[0][c];
        }
        const double n0[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                              e1[0] * e2[1] - e1[1] * e2[0]};
        const double n1[3] = {g1[1] * g2[2] - g1[2] * g2[1], g1[2] * g2[0] - g1[0] * g2[2],
                              g1[0] * g2[1] - g1[1] * g2[0]};
        const double d = n0[0] * n1[0] + n0[1] * n1[1] + n0[2] * n1[2];
        if (!(d > 0.0)) return false;
    }
    return true;
}

struct EvalArgs {
    const double* P;
    const double* Q;
    const int32_t* F;
    const uint32_t *off, *adj, *noff, *bnd;
    const int32_t* nbr;
    const int32_t* E;
    const uint32_t* n_edges;  // device count
    int midpoint;
    uint32_t* bits;     // [cap] float32 cost bits, kNoKey when not collapsible
    uint8_t* faces;     // [cap]
    double* pl;         // [cap][3]
    // optional (edge listing): FP64 cost and validity
    double* cost;
    uint8_t* valid;
};

__global__ void qem_eval_kernel(EvalArgs a) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)*a.n_edges) return;
    const int32_t v0 = a.E[2 * e], v1 = a.E[2 * e + 1];
    const uint32_t b0 = a.off[v0], n0 = a.off[v0 + 1] - b0;
    const uint32_t b1 = a.off[v1], n1 = a.off[v1 + 1] - b1;
    const uint32_t r0 = a.noff[v0], m0 = a.noff[v0 + 1] - r0;
    const uint32_t r1 = a.noff[v1], m1 = a.noff[v1 + 1] - r1;
    // faces on the edge: v1's entry in v0's ring (seven stands for more)
    uint32_t c = 0;
    for (uint32_t i = 0; i < m0; ++i) {
        const int32_t code = a.nbr[r0 + i];
        if ((code >> 3) == v1) {
            c = (uint32_t)(code & 7);
            break;
        }
    }
    bool ok = c >= 1 && c <= 2;
    double p[3] = {0.0, 0.0, 0.0}, cost = 0.0;
    if (ok) {
        // link condition over the sorted rings
        uint32_t i = 0, j = 0, common = 0;
        while (i < m0 && j < m1) {
            const int32_t x = a.nbr[r0 + i] >> 3, y = a.nbr[r1 + j] >> 3;
            if (x == y) {
                ++common;
                ++i;
                ++j;
            } else if (x < y) {
                ++i;
            } else {
                ++j;
            }
        }
        if (common != c) ok = false;
        if (m0 == 3 && m1 == 3) ok = false;
    }
    const bool bv0 = a.bnd[v0] != 0, bv1 = a.bnd[v1] != 0, bedge = c == 1;
    if (ok && !bedge && bv0 && bv1) ok = false;
    if (ok) {
        double q[10];
        const double* q0 = a.Q + 10 * (int64_t)v0;
        const double* q1 = a.Q + 10 * (int64_t)v1;
        for (int k = 0; k < 10; ++k) q[k] = q0[k] + q1[k];
        const double* p0 = a.P + 3 * (int64_t)v0;
        const double* p1 = a.P + 3 * (int64_t)v1;
        if (bedge) {
            const double e0 = qerr(q, p0), e1 = qerr(q, p1);
            const double* src = e1 < e0 ? p1 : p0;
            p[0] = src[0];
            p[1] = src[1];
            p[2] = src[2];
        } else if (bv0) {
            p[0] = p0[0];
            p[1] = p0[1];
            p[2] = p0[2];
        } else if (bv1) {
            p[0] = p1[0];
            p[1] = p1[1];
            p[2] = p1[2];
        } else {
            double t = 0.5;
            if (!a.midpoint) {
                const double det = q[0] * (q[4] * q[7] - q[5] * q[5]) - q[1] * (q[1] * q[7] - q[5] * q[2]) +
                                   q[2] * (q[1] * q[5] - q[4] * q[2]);
                const double tr = q[0] + q[4] + q[7];
                if (det > 1e-8 * tr * tr * tr) {
                    const double i00 = q[4] * q[7] - q[5] * q[5], i01 = q[2] * q[5] - q[1] * q[7];
                    const double i02 = q[1] * q[5] - q[2] * q[4], i11 = q[0] * q[7] - q[2] * q[2];
                    const double i12 = q[1] * q[2] - q[0] * q[5], i22 = q[0] * q[4] - q[1] * q[1];
                    double x[3];
                    x[0] = -(i00 * q[3] + i01 * q[6] + i02 * q[8]) / det;
                    x[1] = -(i01 * q[3] + i11 * q[6] + i12 * q[8]) / det;
                    x[2] = -(i02 * q[3] + i12 * q[6] + i22 * q[8]) / det;
                    const double d[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
                    const double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                    if (dd > 0.0) {
                        t = ((x[0] - p0[0]) * d[0] + (x[1] - p0[1]) * d[1] + (x[2] - p0[2]) * d[2]) / dd;
                        if (!(t > 0.0)) t = 0.0;
                        if (t > 1.0) t = 1.0;
                    } else {
                        t = 0.0;
                    }
                }
            }
            for (int k = 0; k < 3; ++k) p[k] = (1.0 - t) * p0[k] + t * p1[k];
        }
        const double E = qerr(q, p);
        if (E == E) {
            cost = E > 0.0 ? E : 0.0;
            const double m0[3] = {p0[0], p0[1], p0[2]}, m1[3] = {p1[0], p1[1], p1[2]};
            ok = no_fold(a.P, a.F, a.adj, b0, n0, v0, v1, m0, p) && no_fold(a.P, a.F, a.adj, b1, n1, v1, v0, m1, p);
        } else {
            ok = false;
        }
    }
    a.bits[e] = ok ? f32_bits(cost) : kNoKey;
    a.faces[e] = (uint8_t)c;
    a.pl[3 * e] = p[0];
    a.pl[3 * e + 1] = p[1];
    a.pl[3 * e + 2] = p[2];
    if (a.cost) a.cost[e] = cost;
    if (a.valid) a.valid[e] = ok ? 1 : 0;
}

// ---- round selection ------------------------------------------------------

// Selection state of the k-th smallest cost bits, rebuilt by every block from
// the digit histograms of the levels above: wave 0 walks the levels.
struct Select {
    uint32_t prefix;  // digits chosen so far
    uint32_t rem;     // rank still to find within the chosen prefix (1-based)
    uint32_t n_valid;
};

// One level: the digit d where the running count first reaches rem.
__device__ void select_level(const uint32_t* __restrict__ h, uint32_t* prefix, uint32_t* rem) {
    const int lane = threadIdx.x & 63;
    uint32_t c[4], s = 0;
    for (int k = 0; k < 4; ++k) {
        c[k] = h[4 * lane + k];
        s += c[k];
    }
    // inclusive scan of the lane sums
    uint32_t inc = s;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    const uint32_t before = inc - s;
    const bool mine = before < *rem && *rem <= inc;
    const uint64_t bal = __ballot(mine);
    const int src = __ffsll((unsigned long long)bal) - 1;
    uint32_t digit = 0, r = *rem - before;
    if (mine) {
        uint32_t acc = 0;
        for (int k = 0; k < 4; ++k) {
            if (r <= acc + c[k]) {
                digit = 4 * lane + k;
                r -= acc;
                break;
            }
            acc += c[k];
        }
    }
    digit = __shfl(digit, src, 64);
    r = __shfl(r, src, 64);
    *prefix = (*prefix << 8) | digit;
    *rem = r;
}

__device__ void selection(const uint32_t* __restrict__ hist, int levels, double rho, Select* out) {
    // wave 0 of the block; the caller publishes through LDS
    const int lane = threadIdx.x & 63;
    uint32_t s = 0;
    for (int k = 0; k < 4; ++k) s += hist[4 * lane + k];
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    Select st;
    st.n_valid = s;
    st.prefix = 0;
    if (s == 0) {
        st.rem = 0;
        *out = st;
        return;
    }
    int64_t k = (int64_t)ceil(rho * (double)s);
    if (k < 1) k = 1;
    if (k > (int64_t)s) k = s;
    st.rem = (uint32_t)k;
    for (int l = 0; l < levels; ++l) select_level(hist + 256 * l, &st.prefix, &st.rem);
    *out = st;
}

// Level l histogram of the valid cost bits whose upper digits match the
// prefix chosen from levels 0..l-1.
__global__ void __launch_bounds__(kQB) qem_hist_kernel(const uint32_t* __restrict__ bits,
                                                       const uint32_t* __restrict__ n_edges, int64_t grid_n,
                                                       uint32_t* __restrict__ hist, int level, double rho) {
    __shared__ uint32_t h[256];
    __shared__ uint32_t s_prefix, s_skip;
    h[threadIdx.x] = 0;
    if (threadIdx.x < 64) {
        Select st;
        if (level > 0) {
            selection(hist, level, rho, &st);
        } else {
            st.prefix = 0;
            st.n_valid = 1;
        }
        if (threadIdx.x == 0) {
            s_prefix = st.prefix;
            s_skip = st.n_valid == 0;
        }
    }
    __syncthreads();
    if (s_skip) return;
    const int64_t ne = *n_edges;
    const int shift_hi = 32 - 8 * level, shift = 24 - 8 * level;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += grid_n) {
        const uint32_t x = bits[e];
        if (x == kNoKey) continue;
        if (level > 0 && (x >> shift_hi) != s_prefix) continue;
        atomicAdd(&h[(x >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[256 * level + threadIdx.x], h[threadIdx.x]);
}

// Counter slots of a round
constexpr int kQcEdges = 0, kQcValid = 1, kQcTau = 4, kQcLive = 5, kQcApplied = 6, kQcRemoved = 7, kQcCutLo = 8,
              kQcCutHi = 9, kQcStatus = 10, kQcOut = 11, kQcVerts = 12, kQcSlots = 16;

// m(v): least key of the eligible edges at v.
__global__ void __launch_bounds__(kQB) qem_vmin_kernel(const int32_t* __restrict__ E,
                                                       const uint32_t* __restrict__ bits,
                                                       const uint32_t* __restrict__ hist, uint32_t* __restrict__ cnt,
                                                       double rho, uint64_t* __restrict__ m) {
    __shared__ uint32_t s_tau, s_nvalid;
    if (threadIdx.x < 64) {
        Select st;
        selection(hist, 4, rho, &st);
        if (threadIdx.x == 0) {
            s_tau = st.prefix;
            s_nvalid = st.n_valid;
        }
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        cnt[kQcTau] = s_tau;
        cnt[kQcValid] = s_nvalid;
    }
    if (s_nvalid == 0) return;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)cnt[kQcEdges]) return;
    const uint32_t x = bits[e];
    if (x == kNoKey || x > s_tau) return;
    const unsigned long long key = ((unsigned long long)x << 32) | (unsigned long long)(uint32_t)e;
    atomicMin((unsigned long long*)&m[E[2 * e]], key);
    atomicMin((unsigned long long*)&m[E[2 * e + 1]], key);
}

// M(v): least m over v and its ring (every edge, collapsible or not; M
// starts at all ones and a vertex with an eligible edge has that edge).
__global__ void qem_nmin_kernel(const int32_t* __restrict__ E, const uint32_t* __restrict__ cnt,
                                const uint64_t* __restrict__ m, uint64_t* __restrict__ M) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)cnt[kQcEdges]) return;
    const int32_t a = E[2 * e], b = E[2 * e + 1];
    const uint64_t ma = m[a], mb = m[b];
    const uint64_t lo = ma < mb ? ma : mb;
    if (lo == ~0ull) return;
    if (lo < M[a]) atomicMin((unsigned long long*)&M[a], (unsigned long long)lo);
    if (lo < M[b]) atomicMin((unsigned long long*)&M[b], (unsigned long long)lo);
}

// Winners: flag per edge, and per block the number of winners and the faces
// they would remove (no atomics: a round has tens of thousands of winners).
__global__ void __launch_bounds__(kQB) qem_win_kernel(const int32_t* __restrict__ E,
                                                      const uint32_t* __restrict__ bits,
                                                      const uint8_t* __restrict__ faces,
                                                      const uint64_t* __restrict__ M,
                                                      const uint32_t* __restrict__ cnt, uint8_t* __restrict__ wflag,
                                                      uint32_t* __restrict__ part) {
    __shared__ uint32_t s_n[kQB / 64], s_f[kQB / 64];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ne = cnt[kQcEdges];
    bool w = false;
    uint32_t f = 0;
    if (e < ne) {
        const uint32_t x = bits[e];
        if (cnt[kQcValid] != 0 && x != kNoKey && x <= cnt[kQcTau]) {
            const uint64_t key = ((uint64_t)x << 32) | (uint64_t)(uint32_t)e;
            w = M[E[2 * e]] == key && M[E[2 * e + 1]] == key;
            if (w) f = faces[e];
        }
        wflag[e] = w ? 1 : 0;
    }
    uint32_t n = w ? 1u : 0u;
    for (int o = 32; o >= 1; o >>= 1) {
        n += __shfl_xor(n, o, 64);
        f += __shfl_xor(f, o, 64);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_n[wave] = n;
        s_f[wave] = f;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tn = 0, tf = 0;
        for (int k = 0; k < kQB / 64; ++k) {
            tn += s_n[k];
            tf += s_f[k];
        }
        part[2 * blockIdx.x] = tn;
        part[2 * blockIdx.x + 1] = tf;
    }
}

// The collapses a round applies.  Sums the per-block winner counts; when the
// winners would remove more than live - target faces, finds the smallest key
// that no longer fits (keys ascending, face counts summed) by a radix descent
// over the winners' 64-bit keys, 8 bits per level.  Writes the cut key and the
// number of collapses kept and the faces they remove.  One workgroup.
__global__ void __launch_bounds__(1024) qem_cut_kernel(const uint8_t* __restrict__ wflag,
                                                       const uint32_t* __restrict__ bits,
                                                       const uint8_t* __restrict__ faces,
                                                       const uint32_t* __restrict__ part, int64_t nblk,
                                                       uint32_t* __restrict__ cnt, int64_t target) {
    __shared__ uint32_t h[256], hc[256];
    __shared__ uint32_t s_red[2][1024 / 64];
    __shared__ unsigned long long s_prefix;
    __shared__ uint32_t s_budget, s_kf, s_kn;
    uint32_t n = 0, f = 0;
    for (int64_t i = threadIdx.x; i < nblk; i += blockDim.x) {
        n += part[2 * i];
        f += part[2 * i + 1];
    }
    for (int o = 32; o >= 1; o >>= 1) {
        n += __shfl_xor(n, o, 64);
        f += __shfl_xor(f, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_red[0][threadIdx.x >> 6] = n;
        s_red[1][threadIdx.x >> 6] = f;
    }
    __syncthreads();
    uint32_t tn = 0, tf = 0;
    for (int k = 0; k < 1024 / 64; ++k) {
        tn += s_red[0][k];
        tf += s_red[1][k];
    }
    const int64_t budget = (int64_t)cnt[kQcLive] - target;
    if ((int64_t)tf <= budget) {
        if (threadIdx.x == 0) {
            cnt[kQcCutLo] = 0xFFFFFFFFu;
            cnt[kQcCutHi] = 0xFFFFFFFFu;
            cnt[kQcApplied] = tn;
            cnt[kQcRemoved] = tf;
        }
        return;
    }
    const int64_t ne = cnt[kQcEdges];
    if (threadIdx.x == 0) {
        s_prefix = 0;
        s_budget = (uint32_t)(budget > 0 ? budget : 0);
        s_kf = 0;
        s_kn = 0;
    }
    for (int level = 0; level < 8; ++level) {
        const int shift = 56 - 8 * level;
        if (threadIdx.x < 256) {
            h[threadIdx.x] = 0;
            hc[threadIdx.x] = 0;
        }
        __syncthreads();
        const unsigned long long pre = s_prefix;
        for (int64_t e = threadIdx.x; e < ne; e += blockDim.x) {
            if (!wflag[e]) continue;
            const uint64_t k = ((uint64_t)bits[e] << 32) | (uint64_t)(uint32_t)e;
            if (level > 0 && (k >> (shift + 8)) != pre) continue;
            atomicAdd(&h[(k >> shift) & 255u], (uint32_t)faces[e]);
            atomicAdd(&hc[(k >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t acc = 0, accn = 0, d = 0;
            for (; d < 256; ++d) {
                if (acc + h[d] > s_budget) break;
                acc += h[d];
                accn += hc[d];
            }
            // the winners under the prefix weigh more than the budget, so a digit overflows
            s_prefix = (pre << 8) | (d < 256 ? d : 255u);
            s_budget -= acc;
            s_kf += acc;
            s_kn += accn;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cnt[kQcCutLo] = (uint32_t)s_prefix;
        cnt[kQcCutHi] = (uint32_t)(s_prefix >> 32);
        cnt[kQcApplied] = s_kn;
        cnt[kQcRemoved] = s_kf;
    }
}

__global__ void qem_apply_kernel(const uint8_t* __restrict__ wflag, const uint32_t* __restrict__ bits,
                                 const int32_t* __restrict__ E, const double* __restrict__ pl,
                                 const uint32_t* __restrict__ cnt, double* __restrict__ P, double* __restrict__ Q,
                                 int32_t* __restrict__ partner) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)cnt[kQcEdges] || !wflag[e]) return;
    const uint64_t cut = ((uint64_t)cnt[kQcCutHi] << 32) | cnt[kQcCutLo];
    const uint64_t key = ((uint64_t)bits[e] << 32) | (uint64_t)(uint32_t)e;
    if (key >= cut) return;
    const int32_t v0 = E[2 * e], v1 = E[2 * e + 1];
    P[3 * (int64_t)v0] = pl[3 * e];
    P[3 * (int64_t)v0 + 1] = pl[3 * e + 1];
    P[3 * (int64_t)v0 + 2] = pl[3 * e + 2];
    for (int k = 0; k < 10; ++k) Q[10 * (int64_t)v0 + k] = Q[10 * (int64_t)v0 + k] + Q[10 * (int64_t)v1 + k];
    partner[v1] = v0;
}

// Start of a round: counters (status kept), histograms, m, M, partners, and
// when the face lists are rebuilt, their degree and cursor arrays.
__global__ void qem_reset_kernel(int64_t nv, uint32_t live, int lists, uint32_t* __restrict__ cnt,
                                 uint32_t* __restrict__ hist, uint64_t* __restrict__ m, uint64_t* __restrict__ M,
                                 int32_t* __restrict__ partner, uint32_t* __restrict__ deg,
                                 uint32_t* __restrict__ cur) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kQcStatus) cnt[i] = 0;
    if (i == kQcLive) cnt[i] = live;
    if (i < 4 * 256) hist[i] = 0;
    if (i < nv) {
        m[i] = ~0ull;
        M[i] = ~0ull;
        partner[i] = -1;
        if (lists) cur[i] = 0;
    }
    if (lists && i <= nv) deg[i] = 0;
}

__global__ void qem_face_flag_kernel(const int32_t* __restrict__ F, int64_t live, const int32_t* __restrict__ partner,
                                     int32_t* __restrict__ F2, uint32_t* __restrict__ keep) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= live) return;
    int32_t x[3];
    for (int k = 0; k < 3; ++k) {
        const int32_t v = F[3 * f + k];
        const int32_t p = partner[v];
        x[k] = p >= 0 ? p : v;
    }
    const bool alive = x[0] != x[1] && x[1] != x[2] && x[0] != x[2];
    keep[f] = alive ? 1u : 0u;
    F2[3 * f] = x[0];
    F2[3 * f + 1] = x[1];
    F2[3 * f + 2] = x[2];
}

__global__ void qem_face_scatter_kernel(const int32_t* __restrict__ F2, int64_t live, const uint32_t* __restrict__ keep,
                                        const uint32_t* __restrict__ koff, int32_t* __restrict__ F) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= live || !keep[f]) return;
    const int64_t o = koff[f];
    F[3 * o] = F2[3 * f];
    F[3 * o + 1] = F2[3 * f + 1];
    F[3 * o + 2] = F2[3 * f + 2];
}

// ---- renumbering -----------------------------------------------------------
// Once most vertices are gone, the survivors are renumbered in their order
// (new index = rank among the vertices a live face references): the edge
// order, the keys and the lower-index rule are unchanged, and the per-vertex
// passes of later rounds cover only the survivors.

__global__ void qem_vmove_kernel(const double* __restrict__ P, const double* __restrict__ Q, int64_t nv,
                                 const uint32_t* __restrict__ ref, const uint32_t* __restrict__ vid,
                                 double* __restrict__ P2, double* __restrict__ Q2) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv || !ref[v]) return;
    const int64_t o = vid[v];
    for (int k = 0; k < 3; ++k) P2[3 * o + k] = P[3 * v + k];
    for (int k = 0; k < 10; ++k) Q2[10 * o + k] = Q[10 * v + k];
}

__global__ void qem_frenum_kernel(int32_t* __restrict__ F, int64_t live, const uint32_t* __restrict__ vid) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= live) return;
    for (int k = 0; k < 3; ++k) F[3 * f + k] = (int32_t)vid[F[3 * f + k]];
}

// ---- output ---------------------------------------------------------------

__global__ void qem_ref_kernel(const int32_t* __restrict__ F, int64_t live, uint32_t* __restrict__ ref) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= live) return;
    for (int k = 0; k < 3; ++k) ref[F[3 * f + k]] = 1u;
}

__global__ void qem_vout_kernel(const double* __restrict__ P, int64_t nv, const uint32_t* __restrict__ ref,
                                const uint32_t* __restrict__ vid, float* __restrict__ V_out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv || !ref[v]) return;
    const int64_t o = vid[v];
    V_out[3 * o] = (float)P[3 * v];
    V_out[3 * o + 1] = (float)P[3 * v + 1];
    V_out[3 * o + 2] = (float)P[3 * v + 2];
}

__global__ void qem_fout_kernel(const int32_t* __restrict__ F, int64_t live, const uint32_t* __restrict__ vid,
                                int32_t* __restrict__ F_out) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= live) return;
    for (int k = 0; k < 3; ++k) F_out[3 * f + k] = (int32_t)vid[F[3 * f + k]];
}

__global__ void qem_edge_out_kernel(const int32_t* __restrict__ E, const uint8_t* __restrict__ faces,
                                    const double* __restrict__ pl, const uint32_t* __restrict__ n_edges, int64_t cap,
                                    int32_t* __restrict__ E_out, int32_t* __restrict__ faces_out,
                                    double* __restrict__ p_out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)*n_edges || e >= cap) return;
    E_out[2 * e] = E[2 * e];
    E_out[2 * e + 1] = E[2 * e + 1];
    faces_out[e] = faces[e];
    for (int k = 0; k < 3; ++k) p_out[3 * e + k] = pl[3 * e + k];
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

size_t qem_layout(int64_t nv, int64_t nf, QemLayout* L) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const int64_t cap = 3 * nf + 1;              // edges: every edge has a face, every face three edges
    const int64_t nbr_cap = 6 * nf + 1;          // ring entries: two per face corner at most
    const int64_t scan_n = std::max<int64_t>(std::max<int64_t>(nv, nf), cap) + 1;
    L->nv = nv;
    L->nf = nf;
    L->edge_cap = cap;
    L->cnt = take(4 * kQcSlots);
    L->hist = take(4 * 256 * 4);
    L->P = take(24 * (size_t)nv);
    L->Q = take(80 * (size_t)nv);
    L->P2 = take(24 * (size_t)nv);
    L->Q2 = take(80 * (size_t)nv);
    L->F = take(12 * (size_t)nf);
    L->F2 = take(12 * (size_t)nf);
    L->keep = take(4 * (size_t)nf);
    L->koff = take(4 * (size_t)(nf + 1));
    L->deg = take(4 * (size_t)(nv + 1));
    L->off = take(4 * (size_t)(nv + 1));
    L->cur = take(4 * (size_t)nv);
    L->adj = take(4 * 3 * (size_t)nf);
    L->ncnt = take(4 * (size_t)(nv + 1));
    L->noff = take(4 * (size_t)(nv + 1));
    L->hcnt = take(4 * (size_t)(nv + 1));
    L->eoff = take(4 * (size_t)(nv + 1));
    L->bnd = take(4 * (size_t)nv);
    L->nbr = take(4 * (size_t)nbr_cap);
    L->keep_ring = take(4 * (size_t)kRingKeep * (size_t)nv);
    L->E = take(8 * (size_t)cap);
    L->bits = take(4 * (size_t)cap);
    L->faces = take((size_t)cap);
    L->pl = take(24 * (size_t)cap);
    L->m = take(8 * (size_t)nv);
    L->M = take(8 * (size_t)nv);
    L->partner = take(4 * (size_t)nv);
    L->wflag = take((size_t)cap);
    L->part = take(8 * (size_t)blocks_for(cap));
    L->scan_tmp = take(4 * (size_t)(scan_tmp_elems(scan_n) + 1));
    L->total = off;
    return off;
}

namespace {

struct QemPtrs {
    uint32_t *cnt, *hist, *keep, *koff, *deg, *off, *cur, *adj, *ncnt, *noff, *hcnt, *eoff, *bnd, *bits, *scan_tmp;
    double *P, *Q, *P2, *Q2, *pl;
    int32_t *F, *F2, *nbr, *keep_ring, *E, *partner;
    uint8_t *faces, *wflag;
    uint32_t* part;
    uint64_t *m, *M;
};

QemPtrs ptrs(const QemLayout& L, char* ws) {
    QemPtrs p;
    p.cnt = (uint32_t*)(ws + L.cnt);
    p.hist = (uint32_t*)(ws + L.hist);
    p.keep = (uint32_t*)(ws + L.keep);
    p.koff = (uint32_t*)(ws + L.koff);
    p.deg = (uint32_t*)(ws + L.deg);
    p.off = (uint32_t*)(ws + L.off);
    p.cur = (uint32_t*)(ws + L.cur);
    p.adj = (uint32_t*)(ws + L.adj);
    p.ncnt = (uint32_t*)(ws + L.ncnt);
    p.noff = (uint32_t*)(ws + L.noff);
    p.hcnt = (uint32_t*)(ws + L.hcnt);
    p.eoff = (uint32_t*)(ws + L.eoff);
    p.bnd = (uint32_t*)(ws + L.bnd);
    p.bits = (uint32_t*)(ws + L.bits);
    p.scan_tmp = (uint32_t*)(ws + L.scan_tmp);
    p.P = (double*)(ws + L.P);
    p.Q = (double*)(ws + L.Q);
    p.P2 = (double*)(ws + L.P2);
    p.Q2 = (double*)(ws + L.Q2);
    p.pl = (double*)(ws + L.pl);
    p.F = (int32_t*)(ws + L.F);
    p.F2 = (int32_t*)(ws + L.F2);
    p.nbr = (int32_t*)(ws + L.nbr);
    p.keep_ring = (int32_t*)(ws + L.keep_ring);
    p.E = (int32_t*)(ws + L.E);
    p.partner = (int32_t*)(ws + L.partner);
    p.faces = (uint8_t*)(ws + L.faces);
    p.m = (uint64_t*)(ws + L.m);
    p.M = (uint64_t*)(ws + L.M);
    p.wflag = (uint8_t*)(ws + L.wflag);
    p.part = (uint32_t*)(ws + L.part);
    return p;
}

#define QEM_TRY(expr)                        \
    do {                                     \
        hipError_t e_ = (expr);              \
        if (e_ != hipSuccess) return e_;     \
    } while (0)

// vertex -> face lists of the `live` current faces (deg and cur zeroed)
hipError_t build_lists(int64_t nv, const QemPtrs& p, int64_t live, hipStream_t s) {
    hipLaunchKernelGGL(qem_deg_kernel, dim3(blocks_for(live)), dim3(kQB), 0, s, p.F, live, p.deg);
    QEM_TRY(hipGetLastError());
    QEM_TRY(exclusive_scan_u32(p.deg, p.off, nv, p.scan_tmp, p.off + nv, s));
    hipLaunchKernelGGL(qem_adj_kernel, dim3(blocks_for(live)), dim3(kQB), 0, s, p.F, live, p.off, p.cur, p.adj);
    return hipGetLastError();
}

// rings and edges of the current mesh; edge count at cnt[kQcEdges]
hipError_t build_edges(int64_t nv, const QemPtrs& p, hipStream_t s) {
    const int64_t g = nv <= 0 ? 1 : (nv + kRB - 1) / kRB;
    hipLaunchKernelGGL(qem_ring_kernel<false>, dim3(g), dim3(kRB), 0, s, p.F, nv, p.off, p.adj, p.ncnt, p.hcnt,
                       p.bnd, p.noff, p.eoff, p.nbr, p.E, p.keep_ring);
    QEM_TRY(hipGetLastError());
    QEM_TRY(exclusive_scan_u32(p.ncnt, p.noff, nv, p.scan_tmp, p.noff + nv, s));
    QEM_TRY(exclusive_scan_u32(p.hcnt, p.eoff, nv, p.scan_tmp, p.cnt + kQcEdges, s));
    hipLaunchKernelGGL(qem_ring_kernel<true>, dim3(g), dim3(kRB), 0, s, p.F, nv, p.off, p.adj, p.ncnt, p.hcnt,
                       p.bnd, p.noff, p.eoff, p.nbr, p.E, p.keep_ring);
    return hipGetLastError();
}

hipError_t eval_edges(const QemPtrs& p, int64_t edge_grid, int midpoint, double* cost, uint8_t* valid,
                      hipStream_t s) {
    EvalArgs a;
    a.P = p.P;
    a.Q = p.Q;
    a.F = p.F;
    a.off = p.off;
    a.adj = p.adj;
    a.noff = p.noff;
    a.bnd = p.bnd;
    a.nbr = p.nbr;
    a.E = p.E;
    a.n_edges = p.cnt + kQcEdges;
    a.midpoint = midpoint;
    a.bits = p.bits;
    a.faces = p.faces;
    a.pl = p.pl;
    a.cost = cost;
    a.valid = valid;
    hipLaunchKernelGGL(qem_eval_kernel, dim3(blocks_for(edge_grid)), dim3(kQB), 0, s, a);
    return hipGetLastError();
}

hipError_t set_up(const QemLayout& L, const QemPtrs& p, const float* V, const int32_t* F, hipStream_t s) {
    QEM_TRY(fill_u32(p.cnt, 0, kQcSlots, s));
    const int64_t n = std::max(L.nv, L.nf);
    hipLaunchKernelGGL(qem_init_kernel, dim3(blocks_for(n)), dim3(kQB), 0, s, V, L.nv, F, L.nf, p.P, p.partner,
                       p.F, p.cnt + kQcStatus);
    QEM_TRY(hipGetLastError());
    QEM_TRY(fill_u32(p.deg, 0, L.nv + 1, s));
    QEM_TRY(fill_u32(p.cur, 0, L.nv, s));
    QEM_TRY(build_lists(L.nv, p, L.nf, s));
    hipLaunchKernelGGL(qem_quadric_kernel, dim3(blocks_for(L.nv)), dim3(kQB), 0, s, p.P, p.F, L.nv, p.off, p.adj,
                       p.Q);
    return hipGetLastError();
}

}  // namespace

hipError_t qem_edges_run(const QemLayout& L, char* ws, const float* V, const int32_t* F, int midpoint,
                         double* Q_out, int64_t cap, int32_t* E_out, uint8_t* valid_out, int32_t* faces_out,
                         double* cost_out, double* p_out, uint32_t* status, int64_t* n_edges, hipStream_t s) {
    const QemPtrs p = ptrs(L, ws);
    QEM_TRY(set_up(L, p, V, F, s));
    QEM_TRY(build_edges(L.nv, p, s));
    uint32_t h[kQcSlots];
    QEM_TRY(hipMemcpyAsync(h, p.cnt, sizeof h, hipMemcpyDeviceToHost, s));
    QEM_TRY(hipStreamSynchronize(s));
    *status = h[kQcStatus];
    *n_edges = h[kQcEdges];
    if (h[kQcStatus] || (int64_t)h[kQcEdges] > cap) return hipSuccess;
    QEM_TRY(eval_edges(p, h[kQcEdges], midpoint, cost_out, valid_out, s));
    hipLaunchKernelGGL(qem_edge_out_kernel, dim3(blocks_for(h[kQcEdges])), dim3(kQB), 0, s, p.E, p.faces, p.pl,
                       p.cnt + kQcEdges, cap, E_out, faces_out, p_out);
    QEM_TRY(hipGetLastError());
    if (Q_out) QEM_TRY(hipMemcpyAsync(Q_out, p.Q, 80 * (size_t)L.nv, hipMemcpyDeviceToDevice, s));
    return hipStreamSynchronize(s);
}

hipError_t qem_simplify_run(const QemLayout& L, char* ws, const float* V, const int32_t* F, int64_t target, double rho,
                            int32_t max_rounds, int midpoint, float* V_out, int32_t* F_out, int64_t* counts,
                            int32_t* rounds_out, int64_t* stats, float* times_ms, uint32_t* status, hipStream_t s) {
    QemPtrs p = ptrs(L, ws);
    // optional timing: the whole call, and the per-edge evaluation launches summed
    static thread_local hipEvent_t tev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (times_ms) {
        for (int k = 0; k < 4; ++k)
            if (!tev[k]) QEM_TRY(hipEventCreate(&tev[k]));
        times_ms[0] = times_ms[1] = 0.f;
        QEM_TRY(hipEventRecord(tev[2], s));
    }
    QEM_TRY(set_up(L, p, V, F, s));
    // the round counts come back every round: into pinned host memory (one
    // buffer per calling thread, kept for the process), which the copy
    // reaches directly instead of through a staging buffer
    static thread_local uint32_t* h = nullptr;
    if (!h) QEM_TRY(hipHostMalloc((void**)&h, 4 * (kQcSlots + 1), hipHostMallocDefault));
    constexpr size_t kCountBytes = 4 * kQcSlots;
    QEM_TRY(hipMemcpyAsync(h, p.cnt, kCountBytes, hipMemcpyDeviceToHost, s));
    QEM_TRY(hipStreamSynchronize(s));
    *status = h[kQcStatus];
    if (h[kQcStatus]) return hipSuccess;
    int64_t nv = L.nv;  // vertex slots in use (shrinks when the survivors are renumbered)
    int64_t live = L.nf;
    int32_t round = 0;
    while (live > target && round < max_rounds) {
        hipLaunchKernelGGL(qem_reset_kernel, dim3(blocks_for(std::max<int64_t>(nv + 1, 4 * 256))), dim3(kQB), 0, s,
                           nv, (uint32_t)live, round > 0 ? 1 : 0, p.cnt, p.hist, p.m, p.M, p.partner, p.deg, p.cur);
        QEM_TRY(hipGetLastError());
        if (round > 0) QEM_TRY(build_lists(nv, p, live, s));
        QEM_TRY(build_edges(nv, p, s));
        const int64_t egrid = 3 * live;
        if (times_ms) QEM_TRY(hipEventRecord(tev[0], s));
        QEM_TRY(eval_edges(p, egrid, midpoint, nullptr, nullptr, s));
        if (times_ms) QEM_TRY(hipEventRecord(tev[1], s));
        const int64_t hgrid = std::min<int64_t>(blocks_for(egrid), 256);  // few blocks: each merges its bins with global atomics
        for (int level = 0; level < 4; ++level) {
            hipLaunchKernelGGL(qem_hist_kernel, dim3(hgrid), dim3(kQB), 0, s, p.bits, p.cnt + kQcEdges,
                               hgrid * kQB, p.hist, level, rho);
            QEM_TRY(hipGetLastError());
        }
        hipLaunchKernelGGL(qem_vmin_kernel, dim3(blocks_for(egrid)), dim3(kQB), 0, s, p.E, p.bits, p.hist, p.cnt,
                           rho, p.m);
        QEM_TRY(hipGetLastError());
        hipLaunchKernelGGL(qem_nmin_kernel, dim3(blocks_for(egrid)), dim3(kQB), 0, s, p.E, p.cnt, p.m, p.M);
        QEM_TRY(hipGetLastError());
        hipLaunchKernelGGL(qem_win_kernel, dim3(blocks_for(egrid)), dim3(kQB), 0, s, p.E, p.bits, p.faces, p.M,
                           p.cnt, p.wflag, p.part);
        QEM_TRY(hipGetLastError());
        hipLaunchKernelGGL(qem_cut_kernel, dim3(1), dim3(1024), 0, s, p.wflag, p.bits, p.faces, p.part,
                           blocks_for(egrid), p.cnt, target);
        QEM_TRY(hipGetLastError());
        hipLaunchKernelGGL(qem_apply_kernel, dim3(blocks_for(egrid)), dim3(kQB), 0, s, p.wflag, p.bits, p.E, p.pl,
                           p.cnt, p.P, p.Q, p.partner);
        QEM_TRY(hipGetLastError());
        hipLaunchKernelGGL(qem_face_flag_kernel, dim3(blocks_for(live)), dim3(kQB), 0, s, p.F, live, p.partner, p.F2,
                           p.keep);
        QEM_TRY(hipGetLastError());
        QEM_TRY(exclusive_scan_u32(p.keep, p.koff, live, p.scan_tmp, p.cnt + kQcOut, s));
        hipLaunchKernelGGL(qem_face_scatter_kernel, dim3(blocks_for(live)), dim3(kQB), 0, s, p.F2, live, p.keep,
                           p.koff, p.F);
        QEM_TRY(hipGetLastError());
        QEM_TRY(hipMemcpyAsync(h, p.cnt, kCountBytes, hipMemcpyDeviceToHost, s));
        QEM_TRY(hipStreamSynchronize(s));
        live = h[kQcOut];
        if (times_ms) {
            float ms = 0.f;
            QEM_TRY(hipEventElapsedTime(&ms, tev[0], tev[1]));
            times_ms[0] += ms;
        }
        if (stats) {
            stats[4 * round] = h[kQcEdges];
            stats[4 * round + 1] = h[kQcValid];
            stats[4 * round + 2] = h[kQcApplied];
            stats[4 * round + 3] = live;
        }
        ++round;
        if (h[kQcApplied] == 0) break;
        if (live > target && live < nv) {
            // about twice as many slots as live vertices (a closed mesh has
            // about two faces per vertex): renumber the survivors
            uint32_t* ref = p.deg;  // per-round scratch until the next lists
            uint32_t* vid = p.off;
            QEM_TRY(fill_u32(ref, 0, nv + 1, s));
            hipLaunchKernelGGL(qem_ref_kernel, dim3(blocks_for(live)), dim3(kQB), 0, s, p.F, live, ref);
            QEM_TRY(hipGetLastError());
            QEM_TRY(exclusive_scan_u32(ref, vid, nv, p.scan_tmp, p.cnt + kQcVerts, s));
            hipLaunchKernelGGL(qem_vmove_kernel, dim3(blocks_for(nv)), dim3(kQB), 0, s, p.P, p.Q, nv, ref, vid, p.P2,
                               p.Q2);
            QEM_TRY(hipGetLastError());
            hipLaunchKernelGGL(qem_frenum_kernel, dim3(blocks_for(live)), dim3(kQB), 0, s, p.F, live, vid);
            QEM_TRY(hipGetLastError());
            QEM_TRY(hipMemcpyAsync(h + kQcSlots, p.cnt + kQcVerts, 4, hipMemcpyDeviceToHost, s));
            QEM_TRY(hipStreamSynchronize(s));
            nv = h[kQcSlots];
            std::swap(p.P, p.P2);
            std::swap(p.Q, p.Q2);
        }
    }
    *rounds_out = round;
    // output: referenced vertices in ascending index, faces in their order
    uint32_t* ref = p.deg;   // reused: [nv + 1]
    uint32_t* vid = p.off;
    QEM_TRY(fill_u32(ref, 0, nv + 1, s));
    hipLaunchKernelGGL(qem_ref_kernel, dim3(blocks_for(live)), dim3(kQB), 0, s, p.F, live, ref);
    QEM_TRY(hipGetLastError());
    QEM_TRY(exclusive_scan_u32(ref, vid, nv, p.scan_tmp, p.cnt + kQcOut, s));
    hipLaunchKernelGGL(qem_vout_kernel, dim3(blocks_for(nv)), dim3(kQB), 0, s, p.P, nv, ref, vid, V_out);
    QEM_TRY(hipGetLastError());
    hipLaunchKernelGGL(qem_fout_kernel, dim3(blocks_for(live)), dim3(kQB), 0, s, p.F, live, vid, F_out);
    QEM_TRY(hipGetLastError());
    QEM_TRY(hipMemcpyAsync(h, p.cnt, kCountBytes, hipMemcpyDeviceToHost, s));
    if (times_ms) QEM_TRY(hipEventRecord(tev[3], s));
    QEM_TRY(hipStreamSynchronize(s));
    if (times_ms) QEM_TRY(hipEventElapsedTime(&times_ms[1], tev[2], tev[3]));
    counts[0] = h[kQcOut];
    counts[1] = live;
    return hipSuccess;
}

}  // namespace bake
