"""Pins of the oracle's closest-point query (the paper's form of the
correspondence step, Sec. 6.4) against closed forms: orthogonal projection onto
tilted planes with a linear normal field, nearest points on edges and vertices
of a single triangle, the distance filter, a surface baked onto itself, points
off a fine sphere, and brute force against the independent BVH."""
import math

import numpy as np
import pytest

from synth import Asset, make_config
from synth import meshes as M
from planes import grid, plane_asset


def _expected_grid_ids(x, y, V, n):
    xs = V[: n + 1, 0].astype(np.float64)
    j = np.searchsorted(xs, x, side="right") - 1
    i = np.searchsorted(xs, y, side="right") - 1
    x0, x1 = xs[j], xs[j + 1]
    y0, y1 = xs[i], xs[i + 1]
    side = (x1 - x0) * (y - y0) - (y1 - y0) * (x - x0)
    margin = np.minimum.reduce([x - x0, x1 - x, y - y0, y1 - y, np.abs(side) / (x1 - x0)])
    return 2 * (i * n + j) + (side > 0), margin


@pytest.mark.parametrize("s,r,c", [(0.0, 0.0, 0.04), (0.3, -0.2, 0.01), (-0.25, 0.15, -0.08)])
def test_tilted_plane_projection_closed_form(oracle_lib, s, r, c):
    """p = (x, y, 0) above the plane z = s x + r y + c: the closest point is the
    orthogonal projection, at distance |s x + r y + c| / sqrt(1 + s^2 + r^2);
    the normal field (a x, b y, 1) interpolates exactly (it is linear)."""
    oracle = oracle_lib
    n = 9
    V, F = grid(n, z=lambda x, y: s * x + r * y + c, x0=-0.25, y0=-0.25, size=1.5)
    a_, b_ = 0.7, -0.4
    N = np.stack([a_ * V[:, 0], b_ * V[:, 1], np.ones(V.shape[0], np.float32)], 1).astype(np.float32)
    asset = plane_asset(V, F, N, res=64, lo_n=8, max_dist=0.5)
    b = oracle.bake(asset, kind="closest")
    x, y = b.P[:, 0], b.P[:, 1]
    k = math.sqrt(1 + s * s + r * r)
    h = s * x + r * y + c
    assert np.all(b.hit >= 0)
    # float32 vertices; a near-tie neighbour may be up to one quantum farther
    w = 0.5 * 2.0 ** -20
    assert np.abs(b.t - np.abs(h) / k).max() < 2e-7 + w
    # the plane is f = s x + r y - z + c = 0 with gradient (s, r, -1):
    # q = p - f(p) (s, r, -1) / k^2
    qx = x - s * h / (k * k)
    qy = y - r * h / (k * k)
    exp, margin = _expected_grid_ids(qx, qy, V, n)
    # a neighbour at in-plane distance m from the projection is farther by
    # about m^2 / (2 dist): beyond the distance quantum w (where the lower
    # index would win a near tie) once m > sqrt(2 dist w) ~ 4e-4 here
    clear = margin > 1e-3
    assert clear.sum() > 0.9 * clear.size
    assert np.array_equal(b.hit[clear], exp[clear])
    assert np.abs(b.t - np.abs(h) / k)[clear].max() < 2e-7
    # flat lo grid: frame = (x, y, z), so the map is the unit interpolated
    # normal at q (near-tie texels take a neighbour's edge point instead)
    hq = np.stack([a_ * qx, b_ * qy, np.ones_like(qx)], 1)
    hq /= np.linalg.norm(hq, axis=1, keepdims=True)
    assert np.abs(b.map_raw[b.texels][clear] - hq[clear]).max() < 2e-6


def _one_triangle():
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
    F = np.array([[0, 1, 2]], np.int32)
    return V, F


@pytest.mark.parametrize("p,dist,w", [
    ((0.25, 0.25, 0.3), 0.3, (0.5, 0.25, 0.25)),             # projection inside
    ((0.5, -0.4, 0.3), 0.5, (0.5, 0.5, 0.0)),                # nearest on edge v0 v1
    ((0.8, 0.8, 0.1), math.sqrt(0.19), (0.0, 0.5, 0.5)),     # nearest on edge v1 v2
    ((-0.2, 0.5, -0.1), math.sqrt(0.05), (0.5, 0.0, 0.5)),   # nearest on edge v2 v0
    ((-0.3, -0.4, 0.0), 0.5, (1.0, 0.0, 0.0)),               # vertex v0
    ((2.0, -1.0, 0.0), math.sqrt(2.0), (0.0, 1.0, 0.0)),     # vertex v1
    ((-0.5, 1.5, 0.5), math.sqrt(0.75), (0.0, 0.0, 1.0)),    # vertex v2
])
def test_single_triangle_regions(oracle_lib, p, dist, w):
    V, F = _one_triangle()
    P = np.array([p], np.float64)
    for method in ("brute", "bvh"):
        ids, d, ww = oracle_lib.closest(V, F, P, 10.0, method=method)
        assert ids[0] == 0
        assert abs(d[0] - dist) < 1e-12
        assert np.allclose(ww[0], w, atol=1e-12)
    assert abs(oracle_lib.closest_check(V, F, P, np.array([0], np.int32))[0] - dist) < 1e-12


def test_distance_filter_is_inclusive(oracle_lib):
    V, F = _one_triangle()
    P = np.array([[0.25, 0.25, 0.3], [0.25, 0.25, -0.3]])
    ids, _, _ = oracle_lib.closest(V, F, P, 0.3)
    assert np.all(ids == 0)
    ids, _, _ = oracle_lib.closest(V, F, P, 0.3 * (1 - 1e-9))
    assert np.all(ids == -1)


def test_equal_distance_tie_goes_to_lower_index(oracle_lib):
    # two parallel triangles at z = +0.1 and z = -0.1; the point at z = 0 is
    # equidistant: the lower index wins whichever comes first in the list
    V = np.array([[0, 0, 0.1], [1, 0, 0.1], [0, 1, 0.1], [0, 0, -0.1], [1, 0, -0.1], [0, 1, -0.1]], np.float32)
    for F in (np.array([[0, 1, 2], [3, 4, 5]], np.int32), np.array([[3, 4, 5], [0, 1, 2]], np.int32)):
        P = np.array([[0.2, 0.3, 0.0], [0.2, 0.3, 0.01], [0.2, 0.3, -0.01]])
        for method in ("brute", "bvh"):
            ids, d, _ = oracle_lib.closest(V, F, P, 1.0, method=method)
            assert ids[0] == 0
            up = 0 if F[0, 0] == 0 else 1  # index of the z = +0.1 triangle
            assert ids[1] == up and ids[2] == 1 - up
            assert abs(d[0] - 0.1) < 1e-8


def test_surface_baked_onto_itself_is_z(oracle_lib):
    """hi = lo (icosphere level 2) with hi_N = the area-weighted vertex normals:
    every texel position lies on the surface (distance 0), its closest point is
    itself, and the interpolated normal equals d, so the map is (0,0,1)."""
    V, F = M.icosphere(2)
    V = V.astype(np.float32)
    F = F.astype(np.int32)
    N = M.vertex_normals(V.astype(np.float64), F)
    a = Asset("self", V, F, N, V, F, M.face_grid_atlas(F.shape[0], 128), res=128, max_dist=0.01)
    b = oracle_lib.bake(a, kind="closest")
    assert np.all(b.hit >= 0)
    assert b.t.max() < 1e-7
    ang = np.arccos(np.clip(b.map_raw[b.texels][:, 2], -1, 1))
    assert ang.max() < 1e-6
    # away from the face borders the texel's own face is the closest
    inner = b.bary[b.texels].min(1) > 1e-4
    assert inner.sum() > 0.8 * inner.size
    assert np.array_equal(b.hit[inner], b.face[b.texels][inner])


def test_points_off_a_fine_sphere(oracle_lib):
    """p = 1.1 u for unit u, against the level-5 icosphere (chords inside the
    unit sphere): the distance is 0.1 plus at most the chord sag, and the
    closest point lies within a face's width of the radial direction."""
    hV, hF = M.icosphere(5)
    rng = np.random.default_rng(4)
    u = rng.normal(size=(3000, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    P = 1.1 * u
    ids, d, w = oracle_lib.closest(hV.astype(np.float32), hF.astype(np.int32), P, 0.2, method="bvh")
    assert np.all(ids >= 0)
    edge = np.linalg.norm(hV[hF[:, 0]] - hV[hF[:, 1]], axis=1).max()
    sag = 1 - math.sqrt(1 - (edge / math.sqrt(3)) ** 2)  # circumradius of the largest face
    assert d.min() >= 0.1 - 1e-7 and d.max() <= 0.1 + sag + 1e-7
    q = np.einsum("nk,nkj->nj", w, hV[hF[ids]])
    cosang = np.einsum("ij,ij->i", q / np.linalg.norm(q, axis=1, keepdims=True), u)
    assert np.arccos(np.clip(cosang, -1, 1)).max() < edge


def _soup(n, seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(-1, 1, size=(n, 3))
    V = (c[:, None, :] + 0.15 * rng.normal(size=(n, 3, 3))).reshape(-1, 3).astype(np.float32)
    F = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    F[1::3, 0] = F[0::3, 1][: F[1::3].shape[0]]
    return V, F


@pytest.mark.parametrize("seed", [0, 1])
def test_bvh_equals_brute_force_soup(oracle_lib, seed):
    V, F = _soup(3000, seed)
    # a few degenerate triangles (zero area): only their edges count
    F[5] = [F[5, 0], F[5, 0], F[5, 1]]
    rng = np.random.default_rng(200 + seed)
    P = rng.uniform(-1.2, 1.2, size=(4000, 3))
    i1, d1, w1 = oracle_lib.closest(V, F, P, 0.1, method="brute")
    i2, d2, w2 = oracle_lib.closest(V, F, P, 0.1, method="bvh")
    assert (i1 >= 0).sum() > 1000 and (i1 < 0).sum() > 100
    assert np.array_equal(i1, i2) and np.array_equal(d1, d2) and np.array_equal(w1, w2)
    # the winner's distance is the minimum over all triangles (brute check)
    sub = np.nonzero(i1 >= 0)[0][:200]
    for r in sub:
        dd = oracle_lib.closest_check(V, F, np.repeat(P[r:r + 1], F.shape[0], 0), np.arange(F.shape[0], dtype=np.int32))
        assert d1[r] <= dd.min() + 0.1 * 2.0 ** -20


def test_bvh_equals_brute_force_bake_cfg1(oracle_lib):
    a = make_config(1)
    b1 = oracle_lib.bake(a, method="brute", kind="closest")
    b2 = oracle_lib.bake(a, method="bvh", kind="closest")
    assert np.array_equal(b1.hit, b2.hit) and np.array_equal(b1.map, b2.map)
    assert (b1.hit >= 0).sum() > 4000


def test_near_ties_marked(oracle_lib):
    """Two parallel triangles at heights 0.1 and 0.1 + g above a point: a near
    tie when 0 < g <= delta, none when g > delta or when the only other
    triangle shares the nearest point exactly (a fan around a vertex)."""
    delta = 1e-6
    P = np.array([[0.2, 0.2, 0.0]])
    for g, near in ((0.5e-6, True), (3e-6, False)):
        z2 = 0.1 + g
        V = np.float32([[-1, -1, 0.1], [3, -1, 0.1], [-1, 3, 0.1], [-1, -1, z2], [3, -1, z2], [-1, 3, z2]])
        F = np.int32([[0, 1, 2], [3, 4, 5]])
        ids, d, _ = oracle_lib.closest(V, F, P, 1.0)
        assert ids[0] == 0
        assert oracle_lib.closest_near(V, F, P, ids, d, delta).tolist() == [near], g
    # a fan of four triangles around the vertex (0, 0, 0.1) right above the
    # point: every triangle's nearest point is that vertex, an exact tie
    V = np.float32([[0, 0, 0.1], [1, 0, 0.1], [0, 1, 0.1], [-1, 0, 0.1], [0, -1, 0.1]])
    F = np.int32([[0, 1, 2], [0, 2, 3], [0, 3, 4], [0, 4, 1]])
    P = np.array([[0.0, 0.0, -0.2]])
    ids, d, _ = oracle_lib.closest(V, F, P, 1.0)
    assert ids[0] == 0 and abs(d[0] - 0.3) < 1e-7
    assert oracle_lib.closest_near(V, F, P, ids, d, delta).tolist() == [False]
