"""The parity comparator itself, on the CPU: it accepts what FP32 noise can
explain and rejects planted mistakes.  Every "GPU" result here is an oracle
result with one mistake planted in it (the oracle is never changed)."""
import numpy as np
import pytest

from compare import check_first_hits, compare, compare_plain
from synth import Asset, make_config
from synth import meshes as M


@pytest.fixture(scope="module")
def ripple(oracle_lib):
    a = make_config(1)
    return a, oracle_lib.bake(a), oracle_lib.bake(a, rule="plain")


def _as_gpu(ob):
    return ob.map.copy(), ob.status.copy()


def _edge_texels(oracle_lib, a, ob, k=3):
    """Covered texels whose ray crosses a shared high-poly edge (the oracle's
    pick has a weight within 1e-6 of 0 and another face within 1e-9 in distance)."""
    hit = np.nonzero(ob.hit >= 0)[0]
    _, _, bm = oracle_lib.plane_check(a.hi_V, a.hi_F, ob.P[hit], ob.D[hit], ob.hit[hit])
    on = hit[np.abs(bm) < 1e-6]
    out = []
    for r in on:
        ids, t, _ = oracle_lib.query(a.hi_V, a.hi_F, ob.P[r:r + 1], ob.D[r:r + 1], a.max_dist,
                                     exclude=ob.hit[r:r + 1])
        if ids[0] >= 0 and abs(abs(t[0]) - abs(ob.t[r])) < 1e-9:
            out.append(r)
        if len(out) == k:
            break
    assert len(out) == k
    return np.array(out)


def test_oracle_bake_passes_against_itself(oracle_lib, ripple):
    a, ob, _ = ripple
    gm, gh = _as_gpu(ob)
    rep = compare(oracle_lib, a, ob, gm, gh)
    assert rep.ok() and rep.agree == 1.0, str(rep)


def test_plain_rule_bake_is_all_ties_under_the_robust_check(oracle_lib, ripple):
    """The plain rule's picks differ from the robust rule's on 1.2 % of the
    ripple's texels, all at shared edges: every one must pass the tie check
    (the agreement bar, 99.9 %, is what flags them)."""
    a, ob, obp = ripple
    gm, gh = _as_gpu(obp)
    rep = compare(oracle_lib, a, ob, gm, gh)
    print(rep)
    assert rep.n_disagree > 20 and rep.n_ties == rep.n_disagree
    assert rep.failures == [f"id agreement {rep.agree:.6f} < 0.999"]
    # and the robust bake measured against the plain one: all ties
    rp = compare_plain(oracle_lib, a, obp, ob.map_raw, ob.status)
    print(rp)
    assert rp.ok() and rp.n_disagree == rep.n_disagree and rp.max_dt_rel < 1e-6


def test_planted_leak_at_a_shared_edge_fails(oracle_lib, ripple):
    """A ray through a shared edge of the closed high-poly that misses both
    faces (a watertightness leak) is not a tie: the oracle's runner-up with
    its pick excluded is the other face of the edge."""
    a, ob, _ = ripple
    rows = _edge_texels(oracle_lib, a, ob, k=1)
    gm, gh = _as_gpu(ob)
    tex = ob.texels[rows]
    gh[tex] = -1
    gm[tex] = [0, 0, 1]
    rep = compare(oracle_lib, a, ob, gm, gh)
    print(rep)
    assert rep.agree >= 0.999  # one texel: only the tie check can catch it
    assert not rep.ok() and "non-tie" in rep.failures[0]
    rp = compare_plain(oracle_lib, a, oracle_lib.bake(a, rule="plain"), gm, gh)
    assert not rp.ok()


def test_planted_other_face_at_the_edge_is_a_tie(oracle_lib, ripple):
    """The same rays resolved to the other face of the edge: a tie (equal
    distance, both faces met)."""
    a, ob, _ = ripple
    rows = _edge_texels(oracle_lib, a, ob, k=3)
    gm, gh = _as_gpu(ob)
    for r in rows:
        ids, _, _ = oracle_lib.query(a.hi_V, a.hi_F, ob.P[r:r + 1], ob.D[r:r + 1], a.max_dist,
                                     exclude=ob.hit[r:r + 1])
        gh[ob.texels[r]] = ids[0]
    rep = compare(oracle_lib, a, ob, gm, gh)
    assert rep.ok() and rep.n_disagree == 3 and rep.n_ties == 3, str(rep)


def _two_layers():
    """The ripple high-poly plus a copy scaled by 1.04 (a second surface
    0.04 farther out), max_dist 0.2 so both are in range."""
    a = make_config(1)
    V2 = (a.hi_V * np.float32(1.04)).astype(np.float32)
    hV = np.concatenate([a.hi_V, V2])
    hF = np.concatenate([a.hi_F, a.hi_F + a.hi_V.shape[0]]).astype(np.int32)
    hN = np.concatenate([a.hi_N, a.hi_N])
    return Asset("two_layers", hV, hF, hN, a.lo_V, a.lo_F, a.lo_UV, res=a.res, max_dist=0.2), a.hi_F.shape[0]


def test_planted_farther_layer_fails(oracle_lib):
    a, n_in = _two_layers()
    ob = oracle_lib.bake(a)
    gm, gh = _as_gpu(ob)
    inner = np.nonzero((ob.hit >= 0) & (ob.hit < n_in))[0]
    _, _, bm = oracle_lib.plane_check(a.hi_V, a.hi_F, ob.P[inner], ob.D[inner], ob.hit[inner])
    r = inner[np.argmax(bm)]  # a ray well inside its triangle
    outer, t2, _ = oracle_lib.query(a.hi_V, a.hi_F[n_in:], ob.P[r:r + 1], ob.D[r:r + 1], a.max_dist)
    assert outer[0] >= 0 and abs(t2[0]) > abs(ob.t[r]) + 0.01
    gh[ob.texels[r]] = outer[0] + n_in
    rep = compare(oracle_lib, a, ob, gm, gh)
    print(rep)
    assert not rep.ok() and "non-tie" in rep.failures[0]


def test_planted_nearer_triangle_the_ray_misses_fails(oracle_lib, ripple):
    a, ob, _ = ripple
    gm, gh = _as_gpu(ob)
    r = int(np.nonzero(ob.hit >= 0)[0][10])
    gh[ob.texels[r]] = (ob.hit[r] + 37) % a.hi_F.shape[0]
    rep = compare(oracle_lib, a, ob, gm, gh)
    assert not rep.ok() and "non-tie" in rep.failures[0]


def test_planted_miss_in_the_middle_of_a_face_fails(oracle_lib, ripple):
    a, ob, _ = ripple
    gm, gh = _as_gpu(ob)
    hit = np.nonzero(ob.hit >= 0)[0]
    _, _, bm = oracle_lib.plane_check(a.hi_V, a.hi_F, ob.P[hit], ob.D[hit], ob.hit[hit])
    r = hit[np.argmax(bm)]
    gh[ob.texels[r]] = -1
    rep = compare(oracle_lib, a, ob, gm, gh)
    assert not rep.ok()


def test_range_end_miss_is_a_tie(oracle_lib):
    """A plane at |t| = max_dist exactly: a GPU miss there is within noise."""
    from planes import grid, plane_asset
    V, F = grid(3, z=lambda x, y: 0 * x + np.float32(0.25), x0=-0.05, y0=-0.05, size=1.1)
    N = np.tile(np.float32([0, 0, 1]), (V.shape[0], 1))
    a = plane_asset(V, F, N, res=16, lo_n=2, max_dist=float(np.float32(0.25)))
    ob = oracle_lib.bake(a)
    hit = np.nonzero(ob.hit >= 0)[0]
    assert hit.size > 0.3 * ob.texels.size  # the FP64 t rounds to either side of max_dist
    gm, gh = _as_gpu(ob)
    gh[ob.texels[hit[0]]] = -1
    rep = compare(oracle_lib, a, ob, gm, gh, check_dilation=False)
    assert rep.n_disagree == 1 and rep.n_ties == 1 and rep.failures == [f"id agreement {rep.agree:.6f} < 0.999"]


# ---------------------------------------------------------------------------
# camera rays (hidden-face removal)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def sphere_rays(oracle_lib):
    V, F = M.icosphere(3)
    V = V.astype(np.float32)
    F = F.astype(np.int32)
    eyes = M.sphere_viewpoints(4, [0, 0, 0], 2.5)
    P, D = oracle_lib.camera_rays(eyes, [0, 0, 0], np.tan(np.radians(30)), 64)
    ids, t = oracle_lib.first_hit(V, F, P, D, 5.0, "bvh")
    return V, F, P, D, ids, t


def test_first_hits_pass_against_themselves(oracle_lib, sphere_rays):
    V, F, P, D, ids, t = sphere_rays
    rep = check_first_hits(oracle_lib, V, F, P, D, ids, ids, t, 5.0)
    assert rep.ok() and rep.agree == 1.0


def test_first_hits_planted_leak_fails(oracle_lib, sphere_rays):
    V, F, P, D, ids, t = sphere_rays
    hit = np.nonzero(ids >= 0)[0]
    _, _, bm = oracle_lib.plane_check(V, F, P[hit], D[hit], ids[hit])
    # the ray that passes closest to an edge of the closed sphere, and the one
    # through the middle of a face: a miss is a leak for both
    for r in (hit[np.argmin(np.abs(bm))], hit[np.argmax(bm)]):
        g = ids.copy()
        g[r] = -1
        rep = check_first_hits(oracle_lib, V, F, P, D, g, ids, t, 5.0)
        assert not rep.ok() and "non-tie" in rep.failures[0], (r, bm.min())
    # and the farther (back) face of the sphere instead of the front one
    r = hit[np.argmax(bm)]
    back, tb = oracle_lib.first_hit(V, F, P[r:r + 1], D[r:r + 1], 5.0, "brute", exclude=ids[r:r + 1])
    assert back[0] >= 0 and tb[0] > t[r] + 0.1
    g = ids.copy()
    g[r] = back[0]
    assert not check_first_hits(oracle_lib, V, F, P, D, g, ids, t, 5.0).ok()


def _patch_beside_texel_column(dx):
    """A high-poly quad at z = 0.05 over x in [0.1, x1], y in [0.1, 0.9] whose
    boundary edge x = x1 lies dx short of the texel column x = 8.5 / 16 of a
    16^2 flat low-poly (rays along +z)."""
    from planes import plane_asset
    x1 = np.float32(8.5 / 16 - dx)
    V = np.array([[0.1, 0.1, 0.05], [x1, 0.1, 0.05], [x1, 0.9, 0.05], [0.1, 0.9, 0.05]], np.float32)
    F = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    # tilted normals, so a hit bakes a normal other than the miss value (0,0,1)
    N = np.tile(np.float32([0.3, 0, 1]), (4, 1))
    return plane_asset(V, F, N, res=16, lo_n=2, max_dist=0.25)


def test_hit_grazing_a_boundary_edge_is_a_plain_tie(oracle_lib):
    """Rays passing 5e-7 (about 8 FP32 ulps) outside a boundary edge of the
    high-poly: the plain rule misses, the robust rule's edge tolerance admits
    the triangle (as the GPU does).  Against the plain rule such a hit is a tie
    (the ray grazes the triangle); the same hit planted on rays 0.1 away from
    the edge is not."""
    a = _patch_beside_texel_column(5e-7)
    ob = oracle_lib.bake(a, dilate_passes=0)
    obp = oracle_lib.bake(a, rule="plain", dilate_passes=0)
    graze = (ob.hit >= 0) & (obp.hit < 0)
    assert graze.sum() >= 10, int(graze.sum())
    gm, gh = _as_gpu(ob)
    rp = compare_plain(oracle_lib, a, obp, gm, gh)
    print(rp)
    assert rp.ok() and rp.n_disagree == int(graze.sum()) and rp.max_delta_ulp <= 32
    assert rp.max_angle > 10  # the grazing hits' normals are not the miss value
    # planted: the triangle reported on rays of the column 0.1 farther out
    far = np.nonzero((obp.hit < 0) & np.isclose(obp.P[:, 0], 10.5 / 16))[0]
    assert far.size > 0
    gh2 = gh.copy()
    gh2[obp.texels[far[0]]] = 0
    rp2 = compare_plain(oracle_lib, a, obp, gm, gh2)
    assert not rp2.ok()
