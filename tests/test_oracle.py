"""Pins of the FP64 oracle against facts fixed by geometry and the paper.

Each test checks the oracle against something other than itself: closed forms
(flat and tilted planes, undisplaced sphere), a convergence order (analytic
ripple), a theorem (Pick's lattice count), symmetry, hand-derived stencils, and
an independent search structure (BVH vs brute force).
"""
import math

import numpy as np
import pytest

from synth import Asset, make_config
from synth import meshes as M
from planes import grid, plane_asset, plane_uv


def _frame(oracle, asset, b):
    """Tangent frame (T', B', d) of the baked rays, from the oracle's own
    per-face tangent and handedness."""
    vn, ok = oracle.lo_normals(asset.lo_V, asset.lo_F)
    Tf, _, hf, _ = oracle.face_frames(asset.lo_V, asset.lo_F, asset.lo_UV, asset.res, ok)
    lf = b.face[b.texels]
    d = b.D
    T = Tf[lf] - np.einsum("ij,ij->i", d, Tf[lf])[:, None] * d
    T /= np.linalg.norm(T, axis=1, keepdims=True)
    B = hf[lf][:, None] * np.cross(d, T)
    return T, B, d


# ---------------------------------------------------------------------------
# planes
# ---------------------------------------------------------------------------

def _hi_plane(n, zfn, normal, lo=-0.05, size=1.1):
    V, F = grid(n, z=zfn, x0=lo, y0=lo, size=size)
    N = np.tile(np.asarray(normal, np.float32), (V.shape[0], 1))
    return V, F, N


def _expected_grid_ids(x, y, V, n):
    """Triangle of the hi grid containing (x, y), computed from the float32 grid
    coordinates by cell lookup and the side of the cell diagonal."""
    xs = V[: n + 1, 0].astype(np.float64)
    j = np.searchsorted(xs, x, side="right") - 1
    i = np.searchsorted(xs, y, side="right") - 1
    x0, x1 = xs[j], xs[j + 1]
    y0, y1 = xs[i], xs[i + 1]
    side = (x1 - x0) * (y - y0) - (y1 - y0) * (x - x0)  # > 0 above the diagonal
    margin = np.minimum.reduce([x - x0, x1 - x, y - y0, y1 - y, np.abs(side) / (x1 - x0)])
    return 2 * (i * n + j) + (side > 0), margin


def test_flat_plane_bakes_to_z_with_t_zero(oracle_lib):
    oracle = oracle_lib
    hV, hF, hN = _hi_plane(7, lambda x, y: 0 * x, (0, 0, 1))
    a = plane_asset(hV, hF, hN, res=64, lo_n=8, max_dist=0.25)
    b = oracle.bake(a)
    cov = b.face >= 0
    assert cov.all()  # the lo grid covers the whole atlas
    assert np.all(b.hit >= 0)
    assert np.abs(b.t).max() < 1e-15
    assert np.allclose(b.map_raw, [0, 0, 1], atol=1e-15)
    x, y = b.P[:, 0], b.P[:, 1]
    exp, margin = _expected_grid_ids(x, y, hV, 7)
    # away from the edge tolerance band the containing triangle wins
    clear = margin > 4 * oracle.EDGE_EPS * 1.1 / 7
    assert clear.sum() > 0.9 * clear.size
    assert np.array_equal(b.hit[clear], exp[clear])


@pytest.mark.parametrize("s,r,c", [(0.3, -0.2, 0.01), (-0.25, 0.15, -0.08)])
def test_tilted_plane_closed_form(oracle_lib, s, r, c):
    oracle = oracle_lib
    nrm = np.array([-s, -r, 1.0]) / math.sqrt(1 + s * s + r * r)
    hV, hF, hN = _hi_plane(9, lambda x, y: s * x + r * y + c, nrm)
    a = plane_asset(hV, hF, hN, res=64, lo_n=8, max_dist=0.5)
    b = oracle.bake(a)
    x, y = b.P[:, 0], b.P[:, 1]
    assert np.all(b.hit >= 0)
    # the ray along +z from (x, y, 0) meets the plane at t = s x + r y + c
    assert np.abs(b.t - (s * x + r * y + c)).max() < 2e-7  # float32 vertex z
    assert np.abs(b.map_raw[b.texels] - nrm).max() < 1e-7
    exp, margin = _expected_grid_ids(x, y, hV, 9)
    clear = margin > 4 * oracle.EDGE_EPS * 1.1 / 9
    assert clear.sum() > 0.9 * clear.size
    assert np.array_equal(b.hit[clear], exp[clear])


def test_mirrored_chart_flips_handedness(oracle_lib):
    """UV u = 1 - x: T points along -x and the bitangent still along +y."""
    oracle = oracle_lib
    s, r = 0.3, -0.2
    nrm = np.array([-s, -r, 1.0]) / math.sqrt(1 + s * s + r * r)
    hV, hF, hN = _hi_plane(9, lambda x, y: s * x + r * y, nrm)
    lo_V, lo_F = grid(8)
    uv = plane_uv(lo_V, lo_F)
    uv[:, :, 0] = 1.0 - uv[:, :, 0]
    a = Asset("mirror", hV, hF, hN, lo_V, lo_F, uv, res=64, max_dist=0.5)
    _, ok = oracle.lo_normals(lo_V, lo_F)
    _, _, hf, rel = oracle.face_frames(lo_V, lo_F, uv, 64, ok)
    assert np.all(hf == -1) and rel.all()
    b = oracle.bake(a)
    assert (b.face >= 0).all()
    assert np.abs(b.map_raw[b.texels] - [-nrm[0], nrm[1], nrm[2]]).max() < 1e-7


def test_range_is_inclusive_and_two_sided(oracle_lib):
    oracle = oracle_lib
    md = 0.25
    for c, expect_hit in [(md * (1 - 1e-6), True), (-md * (1 - 1e-6), True),
                          (md * (1 + 1e-6), False), (-md * (1 + 1e-6), False)]:
        hV, hF, hN = _hi_plane(3, lambda x, y: 0 * x + c, (0, 0, 1))
        a = plane_asset(hV, hF, hN, res=16, lo_n=2, max_dist=md)
        b = oracle.bake(a)
        if expect_hit:
            assert np.all(b.hit >= 0)
            assert np.allclose(b.t, np.float32(c), atol=1e-12)
        else:
            assert np.all(b.hit == -1)
            assert np.all(b.status[b.texels] == -1)
            assert np.allclose(b.map_raw, [0, 0, 1])


def test_equal_distance_tie_goes_to_lower_index(oracle_lib):
    oracle = oracle_lib
    c = 0.1
    V1, F1, N1 = _hi_plane(3, lambda x, y: 0 * x + c, (0, 0, 1))
    V2, F2, N2 = _hi_plane(3, lambda x, y: 0 * x - c, (0, 0, 1))
    n1 = F1.shape[0]
    for first_above in (True, False):
        A = (V1, F1) if first_above else (V2, F2)
        B = (V2, F2) if first_above else (V1, F1)
        V = np.concatenate([A[0], B[0]])
        F = np.concatenate([A[1], B[1] + A[0].shape[0]]).astype(np.int32)
        N = np.tile(np.float32([0, 0, 1]), (V.shape[0], 1))
        a = plane_asset(V, F, N, res=16, lo_n=2, max_dist=0.5)
        b = oracle.bake(a)
        assert np.all((b.hit >= 0) & (b.hit < n1))  # the first copy always wins
        assert np.allclose(np.abs(b.t), c)
        assert np.all(np.sign(b.t) == (1 if first_above else -1))


def test_duplicate_triangle_resolves_to_lower_index(oracle_lib):
    oracle = oracle_lib
    hV, hF, hN = _hi_plane(4, lambda x, y: 0.05 + 0 * x, (0, 0, 1))
    dup = np.concatenate([hF, hF]).astype(np.int32)
    perm = np.random.default_rng(0).permutation(dup.shape[0])
    F = dup[perm]
    a = plane_asset(hV, F, hN, res=16, lo_n=2, max_dist=0.5)
    for method in ("brute", "bvh"):
        b = oracle.bake(a, method=method)
        # each hit is the lower of the two indices holding the same triangle
        tri = F[b.hit]
        for k, g in enumerate(b.hit):
            same = np.nonzero((F == tri[k]).all(1))[0]
            assert g == same.min()


# ---------------------------------------------------------------------------
# spheres
# ---------------------------------------------------------------------------

def test_lo_normals_radial_on_level1_icosphere(oracle_lib):
    # every vertex of the level-1 icosphere has a rotational symmetry about its
    # radius, so the area-weighted normal is radial (up to float32 inputs)
    V, F = M.icosphere(1)
    n, ok = oracle_lib.lo_normals(V.astype(np.float32), F.astype(np.int32))
    assert ok.all()
    assert np.abs(n - V).max() < 1e-6


def test_flat_grid_normals_and_frames(oracle_lib):
    V, F = grid(5)
    n, ok = oracle_lib.lo_normals(V, F)
    assert np.abs(n - [0.0, 0, 1]).max() < 1e-15
    T, B, h, rel = oracle_lib.face_frames(V, F, plane_uv(V, F), 64, ok)
    assert rel.all() and np.all(h == 1)
    Tn = T / np.linalg.norm(T, axis=1, keepdims=True)
    Bn = B / np.linalg.norm(B, axis=1, keepdims=True)
    assert np.allclose(Tn, [1, 0, 0]) and np.allclose(Bn, [0, 1, 0])


def test_right_triangle_chart_frames(oracle_lib):
    # chart corner 1 sits at +u and corner 2 at +v from corner 0, so T_f is
    # along V1 - V0 and B_f along V2 - V0; outward faces give h = +1
    a = make_config(1)
    _, ok = oracle_lib.lo_normals(a.lo_V, a.lo_F)
    T, B, h, rel = oracle_lib.face_frames(a.lo_V, a.lo_F, a.lo_UV, a.res, ok)
    V = a.lo_V.astype(np.float64)
    e1 = V[a.lo_F[:, 1]] - V[a.lo_F[:, 0]]
    e2 = V[a.lo_F[:, 2]] - V[a.lo_F[:, 0]]
    cosT = np.einsum("ij,ij->i", T, e1) / np.linalg.norm(T, axis=1) / np.linalg.norm(e1, axis=1)
    cosB = np.einsum("ij,ij->i", B, e2) / np.linalg.norm(B, axis=1) / np.linalg.norm(e2, axis=1)
    assert np.all(cosT > 1 - 1e-12) and np.all(cosB > 1 - 1e-12)
    assert rel.all() and np.all(h == 1)


def test_undisplaced_sphere_bakes_to_z(oracle_lib):
    # lo normals radial => d = p/|p|; the hit q on the hi chord surface is along
    # d; with hi_N = vertex positions the interpolated normal is q/|q| = d
    lV, lF = M.icosphere(1)
    hV, hF = M.icosphere(4)
    a = Asset("sphere", hV.astype(np.float32), hF.astype(np.int32), hV.astype(np.float32),
              lV.astype(np.float32), lF.astype(np.int32), M.face_grid_atlas(80, 128),
              res=128, max_dist=0.1)
    b = oracle_lib.bake(a)
    hit = b.hit >= 0
    assert hit.all()
    ang = np.arccos(np.clip(b.map_raw[b.texels][:, 2], -1, 1))
    assert ang.max() < 2e-6  # radians; float32 inputs
    # a flat face normal instead of the interpolated one would be off by degrees
    assert np.all(b.t > 0) and b.t.max() < 0.1


def test_no_surface_within_range_is_a_miss(oracle_lib):
    lV, lF = M.icosphere(1)
    hV, hF = M.icosphere(3)
    a = Asset("far", (1.5 * hV).astype(np.float32), hF.astype(np.int32), hV.astype(np.float32),
              lV.astype(np.float32), lF.astype(np.int32), M.face_grid_atlas(80, 64), res=64,
              max_dist=0.1)
    b = oracle_lib.bake(a)
    assert np.all(b.status[b.texels] == -1)
    assert np.allclose(b.map_raw, [0, 0, 1])


def _ripple_error(oracle, hi_level, lo_level=2, res=128):
    lV, lF = M.icosphere(lo_level)
    hV, hF = M.icosphere(hi_level)
    U = M.unit_directions(hV)
    hiV = M.displace(U, M.analytic_radius(U))
    hiN = M.analytic_normal(M.unit_directions(hiV))
    pole = np.isnan(hiN).any(1)  # the ripple has a kink at the poles
    hiN[pole] = M.unit_directions(hiV)[pole]
    hiN = hiN.astype(np.float32)
    a = Asset("ripple", hiV, hF.astype(np.int32), hiN, lV.astype(np.float32), lF.astype(np.int32),
              M.face_grid_atlas(lF.shape[0], res), res=res, max_dist=0.15)
    b = oracle.bake(a)
    ok = b.hit >= 0
    T, B, d = _frame(oracle, a, b)
    m = b.map_raw[b.texels]
    nw = m[:, :1] * T + m[:, 1:2] * B + m[:, 2:] * d
    q = b.P + b.t[:, None] * b.D
    uq = q / np.linalg.norm(q, axis=1, keepdims=True)
    th = np.arccos(np.clip(uq[:, 2], -1, 1))
    keep = ok & (th > 0.05) & (th < math.pi - 0.05)
    keep &= ~pole[hF[np.maximum(b.hit, 0)]].any(1)
    na = M.analytic_normal(uq)
    err = np.arccos(np.clip(np.einsum("ij,ij->i", nw, na), -1, 1))
    return err[keep].mean(), keep.sum()


def test_analytic_ripple_converges_second_order(oracle_lib):
    e = [_ripple_error(oracle_lib, L) for L in (3, 4, 5, 6)]
    errs = [x[0] for x in e]
    assert all(n > 1000 for _, n in e)
    ratios = [errs[k] / errs[k + 1] for k in range(3)]
    # piecewise-linear normals on a smooth surface: O(h^2), h halves per level
    assert all(2.8 < q < 5.0 for q in ratios), ratios
    assert errs[-1] < 2e-3


# ---------------------------------------------------------------------------
# BVH == brute force
# ---------------------------------------------------------------------------

def _soup(n, seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(-1, 1, size=(n, 3))
    V = (c[:, None, :] + 0.15 * rng.normal(size=(n, 3, 3))).reshape(-1, 3).astype(np.float32)
    F = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    # shared vertices: reuse some triangles' vertices
    F[1::3, 0] = F[0::3, 1][: F[1::3].shape[0]]
    return V, F


def test_bvh_equals_brute_force_cfg1(oracle_lib):
    a = make_config(1)
    b1 = oracle_lib.bake(a, method="brute")
    b2 = oracle_lib.bake(a, method="bvh")
    assert np.array_equal(b1.hit, b2.hit)
    assert np.array_equal(b1.t, b2.t)
    assert np.array_equal(b1.map, b2.map)
    # (T', B', d) is orthonormal, so every encoded hit normal has unit length
    h = b1.hit >= 0
    assert h.sum() > 4000
    assert np.abs(np.linalg.norm(b1.map_raw[b1.texels][h], axis=1) - 1).max() < 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_bvh_equals_brute_force_soup(oracle_lib, seed):
    V, F = _soup(3000, seed)
    rng = np.random.default_rng(100 + seed)
    P = rng.uniform(-1, 1, size=(4000, 3))
    D = rng.normal(size=(4000, 3))
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    # include axis-aligned directions (zero components)
    D[:300] = np.eye(3)[rng.integers(0, 3, 300)] * rng.choice([-1, 1], (300, 1))
    i1, t1, b1 = oracle_lib.query(V, F, P, D, 0.4, method="brute")
    i2, t2, b2 = oracle_lib.query(V, F, P, D, 0.4, method="bvh")
    assert (i1 >= 0).sum() > 500
    assert np.array_equal(i1, i2) and np.array_equal(t1, t2)


def test_bvh_equals_brute_force_decimated_sphere_with_holes(oracle_lib):
    lV, lF = M.icosphere(2)
    hV, hF = M.icosphere(5)
    U = M.unit_directions(hV)
    hiV = M.displace(U, M.noise_radius(U, 3, 4, 0.03))
    hiV, hiF = M.decimate(hiV, hF, 12000, seed=5)
    hiF = hiF.astype(np.int32)
    a = Asset("holes", hiV, hiF, M.vertex_normals(hiV, hiF), lV.astype(np.float32),
              lF.astype(np.int32), M.face_grid_atlas(lF.shape[0], 128), res=128, max_dist=0.1)
    b1 = oracle_lib.bake(a, method="brute")
    b2 = oracle_lib.bake(a, method="bvh")
    assert (b1.hit == -1).sum() > 100  # holes produce misses
    assert np.array_equal(b1.hit, b2.hit)
    assert np.array_equal(b1.map, b2.map)


# ---------------------------------------------------------------------------
# rasteriser
# ---------------------------------------------------------------------------

def test_raster_counts_of_the_workloads(oracle_lib):
    # covered texel centres of the per-face grid atlas at 128^2 and 2048^2
    f1, _ = oracle_lib.raster(M.face_grid_atlas(80, 128), 128)
    assert (f1 >= 0).sum() == 4233
    f2, _ = oracle_lib.raster(M.face_grid_atlas(20480, 2048), 2048)
    assert (f2 >= 0).sum() == 1082478


def test_raster_pick_theorem(oracle_lib):
    """Triangles with corners on texel centres: covered count (inclusive) is
    I + B = A + B/2 + 1 by Pick's theorem (A in texel^2, B boundary points)."""
    rng = np.random.default_rng(7)
    res = 32
    for _ in range(60):
        P = rng.integers(0, res, size=(3, 2))
        A2 = abs((P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) - (P[2, 0] - P[0, 0]) * (P[1, 1] - P[0, 1]))
        if A2 == 0:
            continue
        Bn = sum(math.gcd(abs(int(P[(k + 1) % 3, 0] - P[k, 0])), abs(int(P[(k + 1) % 3, 1] - P[k, 1])))
                 for k in range(3))
        uv = ((P + 0.5) / res).astype(np.float32)[None]
        if rng.random() < 0.5:
            uv = uv[:, ::-1].copy()  # clockwise corners
        face, bary = oracle_lib.raster(uv, res)
        assert 2 * (face >= 0).sum() == A2 + Bn + 2
        # barycentrics reproduce the texel centre from the snapped corners
        t = np.nonzero(face >= 0)[0]
        X = np.rint(uv[0] * res * 256).astype(np.float64)
        c = bary[t] @ X
        ctr = np.stack([256 * (t % res) + 128, 256 * (t // res) + 128], 1)
        assert np.abs(c - ctr).max() < 1e-9
        assert np.all(bary[t] >= 0) and np.allclose(bary[t].sum(1), 1)


def test_raster_overlap_lowest_face_wins_and_degenerate_uv_covers_nothing(oracle_lib):
    res = 16
    big = np.float32([[[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]])
    small = np.float32([[[0.1, 0.1], [0.5, 0.1], [0.1, 0.5]]])
    line = np.float32([[[0.0, 0.0], [0.5, 0.5], [1.0, 1.0]]])  # zero UV area
    f, _ = oracle_lib.raster(np.concatenate([small, big]), res)
    fs, _ = oracle_lib.raster(small, res)
    assert np.all(f[fs >= 0] == 0)
    f, _ = oracle_lib.raster(np.concatenate([big, small]), res)
    assert np.all(f[f >= 0] == 0)
    f, _ = oracle_lib.raster(line, res)
    assert (f >= 0).sum() == 0


def test_degenerate_lo_face_is_unreliable(oracle_lib):
    lV, lF = grid(2)
    lV = lV.copy()
    F = lF.copy()
    F[3] = [F[3, 0], F[3, 0], F[3, 2]]  # collapsed in 3D, UVs kept
    uv = plane_uv(lV, lF)
    hV, hF, hN = _hi_plane(3, lambda x, y: 0.02 + 0 * x, (0, 0, 1))
    a = Asset("degen", hV, hF, hN, lV, F.astype(np.int32), uv, res=16, max_dist=0.1)
    b = oracle_lib.bake(a)
    bad = b.face == 3
    assert bad.sum() > 0
    assert np.all(b.status[bad] == -2)
    assert np.allclose(b.map_raw[bad], [0, 0, 1])
    assert np.all(b.status[(b.face >= 0) & ~bad] >= 0)


# ---------------------------------------------------------------------------
# dilation, encoding
# ---------------------------------------------------------------------------

def test_dilation_hand_pattern(oracle_lib):
    """4x4 atlas with values a at (0,0) and b at (0,3).  Pass 1 copies a to
    (0,1),(1,0),(1,1) and b to (0,2),(1,2),(1,3); pass 2 gives (2,0)=a,
    (2,1)=n(2a+b), (2,2)=n(a+2b), (2,3)=b; row 3 stays empty."""
    res = 4
    a = np.array([0.6, 0.0, 0.8])
    bb = np.array([0.0, 0.6, 0.8])
    m = np.zeros((16, 3)); m[:, 2] = 1
    lv = np.full(16, 255, np.uint8)
    m[0], lv[0] = a, 0
    m[3], lv[3] = bb, 0
    out, lev = oracle_lib.dilate(m, lv, res, 2)
    n = lambda v: v / np.linalg.norm(v)
    exp = {1: a, 4: a, 5: a, 2: bb, 6: bb, 7: bb, 8: a, 9: n(2 * a + bb), 10: n(a + 2 * bb), 11: bb}
    for t, v in exp.items():
        assert np.allclose(out[t], v, atol=1e-15), t
    assert list(lev[[1, 4, 5, 2, 6, 7]]) == [1] * 6 and list(lev[8:12]) == [2] * 4
    assert np.all(lev[12:] == 255) and np.allclose(out[12:], [0, 0, 1])
    # one pass only touches the first ring
    out1, lev1 = oracle_lib.dilate(m, lv, res, 1)
    assert np.all(lev1[8:] == 255)


def test_dilation_cancelling_neighbours_stay_empty(oracle_lib):
    res = 3
    m = np.zeros((9, 3)); m[:, 2] = 1
    lv = np.full(9, 255, np.uint8)
    m[3], lv[3] = [1, 0, 0], 0
    m[5], lv[5] = [-1, 0, 0], 0
    out, lev = oracle_lib.dilate(m, lv, res, 1)
    assert lev[4] == 255  # zero sum: nothing to normalise


def test_plane_check_on_own_hits(oracle_lib):
    a = make_config(1)
    b = oracle_lib.bake(a)
    hit = b.hit >= 0
    t, dl, bm = oracle_lib.plane_check(a.hi_V, a.hi_F, b.P[hit], b.D[hit], b.hit[hit])
    assert np.abs(t - b.t[hit]).max() < 1e-12
    # the hit rule: every hit's crossing has weights >= -EDGE_EPS and lies
    # within the tolerance band of its triangle
    assert bm.min() >= -oracle_lib.EDGE_EPS
    assert dl.max() < 1e-3 * 0.1
    # a farther triangle's plane is crossed well outside that triangle
    other = (b.hit[hit] + 7) % a.hi_F.shape[0]
    _, dl2, bm2 = oracle_lib.plane_check(a.hi_V, a.hi_F, b.P[hit], b.D[hit], other)
    assert np.median(dl2) > 1e-3 and np.median(bm2) < -1


def _one_tri_rays(xs, z=0.05):
    V = np.float32([[0, 0, z], [1, 0, z], [0, 1, z]])
    F = np.int32([[0, 1, 2]])
    P = np.stack([xs, np.full_like(xs, 0.25), np.zeros_like(xs)], 1)
    D = np.tile([0.0, 0.0, 1.0], (xs.size, 1))
    return V, F, P, D


def test_edge_tolerance_band(oracle_lib):
    """A line crossing the plane at barycentric weight -eps/2 hits, at -2 eps
    misses (the triangle (0,0),(1,0),(0,1): weight of corner 1 is x)."""
    e = oracle_lib.EDGE_EPS
    xs = np.array([0.5, 0.0, -0.5 * e, -0.9 * e, -1.1 * e, -2 * e])
    V, F, P, D = _one_tri_rays(xs)
    for m in ("brute", "bvh"):
        ids, t, beta = oracle_lib.query(V, F, P, D, 0.1, method=m)
        assert ids.tolist() == [0, 0, 0, 0, -1, -1], m
        assert np.allclose(t[:4], np.float32(0.05)) and np.allclose(beta[2:4, 1], xs[2:4])


def test_distance_quantum_tie_rule(oracle_lib):
    """Two parallel triangles: within one distance quantum w the lower index
    wins even when it is slightly farther; a quantum apart the nearer wins."""
    md = 0.25
    w = oracle_lib.t_quantum(md)
    for gap_q, near_wins in [(0.3, False), (2.5, True)]:
        z0 = np.float32(0.1)
        z_far = float(z0) + gap_q * w
        # lower index = the farther plane
        V = np.float32([[-1, -1, z_far], [3, -1, z_far], [-1, 3, z_far],
                        [-1, -1, z0], [3, -1, z0], [-1, 3, z0]])
        F = np.int32([[0, 1, 2], [3, 4, 5]])
        P = np.array([[0.3, 0.3, 0.0]])
        D = np.array([[0.0, 0.0, 1.0]])
        k_near = math.floor(float(z0) / w)
        k_far = math.floor(float(V[0, 2]) / w)
        for m in ("brute", "bvh"):
            ids, t, _ = oracle_lib.query(V, F, P, D, md, method=m)
            exp = 1 if k_near < k_far else 0
            assert ids[0] == exp, (gap_q, m)
        assert (k_near < k_far) == near_wins or gap_q < 1


def test_rgb8(oracle_lib):
    v = np.array([[-1.0, 0.0, 1.0], [-0.999, 0.5, 0.00392]])
    c = oracle_lib.rgb8(v)
    assert c.tolist() == [[0, 128, 255], [0, 191, 128]]
