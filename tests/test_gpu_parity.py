"""GPU parity: the HIP bake (through the C ABI) against the FP64 oracle.

Every test here runs libbake.so's kernels on the GPU and compares with the
oracle on the same seeded inputs (tests/compare.py states the rules).
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from compare import compare, compare_plain, angle_deg  # noqa: E402
from planes import grid, plane_asset, plane_uv  # noqa: E402
from synth import Asset, make_config  # noqa: E402
from synth import meshes as M  # noqa: E402


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_26137_amd.bake as bake
    bake.lib()  # fails loudly if the library was not built
    return bake


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(B, asset, **kw):
    say(f"[gpu] bake {asset.name} res={asset.res} hi={asset.hi_F.shape[0]} lo={asset.lo_F.shape[0]} {kw}")
    t = B.to_device(asset)
    r = B.bake_normals(*t, asset.res, asset.max_dist, **kw)
    torch.cuda.synchronize()
    return r


def np_out(r):
    return r.map.cpu().numpy().reshape(-1, 3), r.hit.cpu().numpy().reshape(-1)


def check(oracle, asset, r, ob=None, method="brute", min_agree=None):
    """Against the oracle's robust rule (the library's convention: the parity
    bar) and its plain rule (every disagreement a tie)."""
    if ob is None:
        ob = oracle.bake(asset, method=method)
    gm, gh = np_out(r)
    rep = compare(oracle, asset, ob, gm, gh)
    say("[gpu]", asset.name, rep)
    assert rep.ok(), str(rep)
    rp = compare_plain(oracle, asset, oracle.bake(asset, method=method, texels=None if ob.texels.size == rep.n_covered
                                                  else ob.texels, rule="plain", dilate_passes=0), gm, gh)
    say("[gpu]", asset.name, rp)
    assert rp.ok(), str(rp)
    assert r.status() == 0
    return rep, ob


# ---------------------------------------------------------------------------
# whole-bake parity
# ---------------------------------------------------------------------------

def test_ripple_config_full(B, oracle_lib):
    a = make_config(1)
    r = run(B, a)
    rep, ob = check(oracle_lib, a, r)
    assert r.ray_count() == 4233
    assert rep.n_compared == 4233


def _hi_plane(n, zfn, normal, lo=-0.05, size=1.1):
    V, F = grid(n, z=zfn, x0=lo, y0=lo, size=size)
    return V, F, np.tile(np.asarray(normal, np.float32), (V.shape[0], 1))


@pytest.mark.parametrize("s,r,c", [(0.0, 0.0, 0.0), (0.3, -0.2, 0.01), (-0.25, 0.15, -0.08)])
def test_planes(B, oracle_lib, s, r, c):
    nrm = np.array([-s, -r, 1.0]) / math.sqrt(1 + s * s + r * r)
    hV, hF, hN = _hi_plane(9, lambda x, y: s * x + r * y + c, nrm)
    a = plane_asset(hV, hF, hN, res=64, lo_n=8, max_dist=0.5)
    res = run(B, a)
    check(oracle_lib, a, res)
    gm, gh = np_out(res)
    assert np.all(gh >= 0)
    assert np.abs(gm - nrm).max() < 2e-6


def test_mirrored_chart(B, oracle_lib):
    s, r = 0.3, -0.2
    nrm = np.array([-s, -r, 1.0]) / math.sqrt(1 + s * s + r * r)
    hV, hF, hN = _hi_plane(9, lambda x, y: s * x + r * y, nrm)
    lo_V, lo_F = grid(8)
    uv = plane_uv(lo_V, lo_F)
    uv[:, :, 0] = 1.0 - uv[:, :, 0]
    a = Asset("mirror", hV, hF, hN, lo_V, lo_F, uv, res=64, max_dist=0.5)
    res = run(B, a)
    check(oracle_lib, a, res)
    gm, _ = np_out(res)
    assert np.abs(gm - [-nrm[0], nrm[1], nrm[2]]).max() < 2e-6


@pytest.mark.parametrize("c,hit", [(0.25 * (1 - 1e-5), True), (-0.25 * (1 - 1e-5), True),
                                   (0.25 * (1 + 1e-5), False), (-0.25 * (1 + 1e-5), False)])
def test_range_ends(B, oracle_lib, c, hit):
    hV, hF, hN = _hi_plane(3, lambda x, y: 0 * x + c, (0, 0, 1))
    a = plane_asset(hV, hF, hN, res=16, lo_n=2, max_dist=0.25)
    res = run(B, a)
    check(oracle_lib, a, res)
    _, gh = np_out(res)
    assert np.all(gh >= 0) if hit else np.all(gh == -1)


def test_two_planes_tie_to_lower_index(B, oracle_lib):
    c = 0.1
    V1, F1, _ = _hi_plane(3, lambda x, y: 0 * x + c, (0, 0, 1))
    V2, F2, _ = _hi_plane(3, lambda x, y: 0 * x - c, (0, 0, 1))
    for first_above in (True, False):
        A = (V1, F1) if first_above else (V2, F2)
        Bm = (V2, F2) if first_above else (V1, F1)
        V = np.concatenate([A[0], Bm[0]])
        F = np.concatenate([A[1], Bm[1] + A[0].shape[0]]).astype(np.int32)
        N = np.tile(np.float32([0, 0, 1]), (V.shape[0], 1))
        a = plane_asset(V, F, N, res=16, lo_n=2, max_dist=0.5)
        res = run(B, a)
        check(oracle_lib, a, res)
        _, gh = np_out(res)
        assert np.all((gh >= 0) & (gh < F1.shape[0]))


def test_duplicate_triangles(B, oracle_lib):
    hV, hF, hN = _hi_plane(4, lambda x, y: 0.05 + 0 * x, (0, 0, 1))
    dup = np.concatenate([hF, hF]).astype(np.int32)
    F = dup[np.random.default_rng(0).permutation(dup.shape[0])]
    a = plane_asset(hV, F, hN, res=16, lo_n=2, max_dist=0.5)
    res = run(B, a)
    rep, _ = check(oracle_lib, a, res)
    assert rep.agree == 1.0


def test_undisplaced_sphere_is_z(B, oracle_lib):
    lV, lF = M.icosphere(1)
    hV, hF = M.icosphere(4)
    a = Asset("sphere", hV.astype(np.float32), hF.astype(np.int32), hV.astype(np.float32),
              lV.astype(np.float32), lF.astype(np.int32), M.face_grid_atlas(80, 128), res=128,
              max_dist=0.1)
    res = run(B, a, dilate_passes=0)
    check(oracle_lib, a, res)
    gm, gh = np_out(res)
    cov = gh != -3
    assert np.all(gh[cov] >= 0)
    assert angle_deg(gm[cov], [0, 0, 1]).max() < 1e-3


def test_holes_and_misses(B, oracle_lib):
    lV, lF = M.icosphere(2)
    hV, hF = M.icosphere(5)
    U = M.unit_directions(hV)
    hiV = M.displace(U, M.noise_radius(U, 3, 4, 0.03))
    hiV, hiF = M.decimate(hiV, hF, 12000, seed=5)
    hiF = hiF.astype(np.int32)
    a = Asset("holes", hiV, hiF, M.vertex_normals(hiV, hiF), lV.astype(np.float32),
              lF.astype(np.int32), M.face_grid_atlas(lF.shape[0], 128), res=128, max_dist=0.1)
    res = run(B, a)
    rep, ob = check(oracle_lib, a, res)
    _, gh = np_out(res)
    assert (gh == -1).sum() > 100


def _noise_asset(hi_level, lo_level, res, seed, max_dist=0.12):
    lV, lF = M.icosphere(lo_level)
    hV, hF = M.icosphere(hi_level)
    U = M.unit_directions(hV)
    hiV = M.displace(U, M.noise_radius(U, seed, 4, 0.03))
    hiF = hF.astype(np.int32)
    return Asset(f"noise_L{hi_level}_L{lo_level}_{res}", hiV, hiF, M.vertex_normals(hiV, hiF),
                 lV.astype(np.float32), lF.astype(np.int32), M.face_grid_atlas(lF.shape[0], res),
                 res=res, max_dist=max_dist)


@pytest.mark.parametrize("hi_level,lo_level,res", [(6, 3, 512), (7, 2, 256)])
def test_noise_multi_tile_brute(B, oracle_lib, hi_level, lo_level, res):
    a = _noise_asset(hi_level, lo_level, res, seed=11)
    r = run(B, a)
    check(oracle_lib, a, r, method="brute")


@pytest.mark.parametrize("passes", [0, 1, 3, 4, 6])
def test_dilation_passes(B, oracle_lib, passes):
    """Every dilation depth against the oracle's (Sec. 6.4 gutters): the fused
    launch (1 to 4 passes, 56-texel tiles with the halo; 256^2 leaves a ragged
    32-texel tail), the per-pass launches (6) and no dilation (0)."""
    a = _noise_asset(6, 3, 256, seed=7)
    r = run(B, a, dilate_passes=passes)
    ob = oracle_lib.bake(a, method="bvh", dilate_passes=passes)
    check(oracle_lib, a, r, ob=ob)
    gm, gh = np_out(r)
    unc = gh == -3
    filled = unc & np.any(gm != np.array([0.0, 0.0, 1.0], np.float32), axis=1)
    o_filled = unc & np.any(ob.map != np.array([0.0, 0.0, 1.0]), axis=1)
    say(f"[gpu] passes={passes}: uncovered {int(unc.sum())}, filled {int(filled.sum())} (oracle {int(o_filled.sum())})")
    assert np.array_equal(filled, o_filled)
    if passes == 0:
        assert not filled.any()
    else:
        assert filled.any()


# ---------------------------------------------------------------------------
# configuration invariance, determinism
# ---------------------------------------------------------------------------

def test_traversal_configs_bitwise_identical(B):
    a = _noise_asset(6, 3, 256, seed=4)
    ref = run(B, a)
    rm, rh = np_out(ref)
    for blk in (64, 128, 256):
        for stk in (8, 16, 32):
            for per in (0, 1, 2, 3):
                r = run(B, a, trav_block=blk, trav_stack=stk, trav_mode=per)
                m, h = np_out(r)
                assert np.array_equal(h, rh), (blk, stk, per)
                assert np.array_equal(m.view(np.uint32), rm.view(np.uint32)), (blk, stk, per)


def test_repeat_is_bitwise_identical(B):
    a = make_config(1)
    r1 = run(B, a)
    m1, h1 = np_out(r1)
    for _ in range(3):
        r2 = run(B, a, workspace=r1.workspace)
        m2, h2 = np_out(r2)
        assert np.array_equal(h1, h2) and np.array_equal(m1.view(np.uint32), m2.view(np.uint32))


# ---------------------------------------------------------------------------
# stages
# ---------------------------------------------------------------------------

def test_raster_bit_exact(B, oracle_lib):
    a = make_config(1)
    r = run(B, a)
    n = r.ray_count()
    rays = r.view(B.VIEW_RAYS).view(torch.int32).cpu().numpy().reshape(-1, 4)[:n]
    face, bary = oracle_lib.raster(a.lo_UV, a.res)
    cov = np.nonzero(face >= 0)[0]
    # face order, then row-major texel order inside the face
    order = np.lexsort((cov, face[cov]))
    exp_tex = cov[order]
    assert np.array_equal(rays[:, 0], exp_tex)
    assert np.array_equal(rays[:, 1], face[exp_tex])
    b = rays[:, 2:].copy().view(np.float32)
    assert np.abs(b - bary[exp_tex][:, 1:]).max() < 1e-6


def test_lo_normals_and_frames(B, oracle_lib):
    a = make_config(1)
    r = run(B, a)
    n = r.view(B.VIEW_LO_N).view(torch.float32).cpu().numpy().reshape(-1, 4)
    on, ok = oracle_lib.lo_normals(a.lo_V, a.lo_F)
    assert np.all(n[:, 3] == 1.0) and ok.all()
    assert np.abs(n[:, :3] - on).max() < 1e-6
    ft = r.view(B.VIEW_FACE_T).view(torch.float32).cpu().numpy().reshape(-1, 4)
    T, _, h, _ = oracle_lib.face_frames(a.lo_V, a.lo_F, a.lo_UV, a.res, ok)
    assert np.array_equal(ft[:, 3].astype(np.int8), h)
    assert angle_deg(ft[:, :3], T).max() < 1e-4


def decode_nodes(raw):
    """Compressed BVH nodes [n, 8] int32 -> decoded child boxes lo, hi [n, 2, 3]
    (float32 arithmetic: the byte times the power-of-two step is exact, the
    add rounds once, as the kernels' fmaf), child refs [n, 2] and the per-axis
    steps [n, 3]."""
    o = raw[:, 0:3].copy().view(np.float32)
    meta = raw[:, 3].copy().view(np.uint32)
    step = np.stack([((meta >> (8 * k)) & 0xFF) << 23 for k in range(3)], 1).astype(np.uint32).view(np.float32)
    qb = raw[:, 4:7].copy().view(np.uint8).reshape(-1, 12).astype(np.float32)
    planes = (qb.reshape(-1, 4, 3) * step[:, None, :] + o[:, None, :]).astype(np.float32)
    lo = np.stack([planes[:, 0], planes[:, 2]], 1)
    hi = np.stack([planes[:, 1], planes[:, 3]], 1)
    child = raw[:, 7].copy().view(np.uint32).astype(np.int64)
    g = (child & ((1 << 30) - 1)).astype(np.int32)
    left = np.where((child >> 30) & 1, ~g, g)
    right = np.where((child >> 31) & 1, ~(g + 1), g + 1)
    return lo, hi, np.stack([left, right], 1).astype(np.int32), step.astype(np.float64)


@pytest.mark.parametrize("hi_level", [6, 8])
def test_sort_is_stable_sort_and_tree_invariants(B, hi_level):
    a = _noise_asset(hi_level, 2, 64, seed=2)
    # poison the workspace so a refit that read a sibling box before it was
    # written would leave NaN or stale values behind
    nbytes = B.workspace_size(a.hi_V.shape[0], a.hi_F.shape[0], a.lo_V.shape[0], a.lo_F.shape[0], a.res)
    ws = torch.full((nbytes,), 255, dtype=torch.uint8, device="cuda")
    r = run(B, a, workspace=ws)
    nf = a.hi_F.shape[0]
    keys = r.view(B.VIEW_SORTED).view(torch.int32).cpu().numpy().view(np.uint32)
    vals = r.view(B.VIEW_SORTED_IDX).view(torch.int32).cpu().numpy()
    assert np.all(np.diff(keys.astype(np.int64)) >= 0)
    eq = keys[1:] == keys[:-1]
    assert np.all(vals[1:][eq] > vals[:-1][eq])          # stable: index order on equal keys
    assert np.array_equal(np.sort(vals), np.arange(nf))   # a permutation
    raw = r.view(B.VIEW_NODES).view(torch.int32).cpu().numpy().reshape(-1, 8)
    lo3, hi3, refs, step = decode_nodes(raw)
    leaves = r.view(B.VIEW_LEAVES).view(torch.float32).cpu().numpy().reshape(-1, 12)
    # every leaf and every non-root internal node is referenced exactly once
    lf = refs[refs < 0]
    assert np.array_equal(np.sort(~lf), np.arange(nf))
    inn = refs[refs >= 0]
    assert np.array_equal(np.sort(inn), np.arange(1, nf - 1))
    tri = leaves[:, :9].reshape(-1, 3, 3)
    tlo, thi = tri.min(1).astype(np.float64), tri.max(1).astype(np.float64)
    ids = leaves[:, 9].copy().view(np.int32)
    assert np.array_equal(np.sort(ids), np.arange(nf))
    assert np.array_equal(tri, a.hi_V[a.hi_F[ids]])
    assert np.isfinite(lo3).all() and np.isfinite(hi3).all()  # every node written (poisoned workspace)
    # the boxes a leaf must have: the triangle bounds widened for the hit
    # rule's edge tolerance (barycentric weights down to -2^-14) by 3 * 2^-14
    # of the extent; subtree boxes are their unions, bottom-up over the levels
    eps = 1.0 / 16384.0
    ext = thi - tlo
    need_lo, need_hi = tlo - 3 * eps * ext, thi + 3 * eps * ext
    levels = [np.array([0])]
    while True:
        c = refs[levels[-1]].reshape(-1)
        c = c[c >= 0]
        if c.size == 0:
            break
        levels.append(c)
    assert sum(x.size for x in levels) == nf - 1
    sub_lo = np.zeros((nf - 1, 3))
    sub_hi = np.zeros((nf - 1, 3))

    def child_box(c):
        blo = np.where((c < 0)[:, None], need_lo[np.where(c < 0, ~c, 0)], sub_lo[np.maximum(c, 0)])
        bhi = np.where((c < 0)[:, None], need_hi[np.where(c < 0, ~c, 0)], sub_hi[np.maximum(c, 0)])
        return blo, bhi

    for lv in reversed(levels):
        for side in (0, 1):
            blo, bhi = child_box(refs[lv, side])
            # the decoded child box contains every triangle below it, widened
            assert np.all(lo3[lv, side] <= blo) and np.all(hi3[lv, side] >= bhi)
            # and is tight to a quantisation step (plus the kernel's own
            # widening of a few 2^-14 of the extent and ulps)
            slack = step[lv] + 4 * eps * (bhi - blo) + 1e-6 * np.maximum(np.abs(blo), np.abs(bhi)) + 1e-30
            assert np.all(lo3[lv, side] >= blo - slack) and np.all(hi3[lv, side] <= bhi + slack)
        l0, h0 = child_box(refs[lv, 0])
        l1, h1 = child_box(refs[lv, 1])
        sub_lo[lv] = np.minimum(l0, l1)
        sub_hi[lv] = np.maximum(h0, h1)
        # the step is about the smallest power of two with 255 steps spanning
        # the node's box (one doubling more where the rounded end falls short)
        span = np.maximum(h0, h1) - np.minimum(l0, l1)
        assert np.all(step[lv] <= np.maximum(4.04 * span / 255, 2.0 ** -125))
    assert np.all(sub_lo[0] <= a.hi_V[a.hi_F].reshape(-1, 3).min(0))


def test_axis_parallel_rays_prune(B):
    """Rays with zero direction components (a flat low-poly: d = (0, 0, 1)
    exactly) must still prune: a slab the ray runs parallel to and outside of
    rejects the box.  Results never depend on this (pruning is conservative);
    the number of box tests does."""
    n = 64
    hV, hF = grid(n, z=lambda x, y: 0.01 + 0.02 * np.sin(7 * x) * np.cos(5 * y), x0=-0.05, y0=-0.05, size=1.1)
    hN = np.tile(np.array([0, 0, 1], np.float32), (hV.shape[0], 1))
    a = plane_asset(hV, hF, hN, res=128, lo_n=8, max_dist=0.25)
    t = B.to_device(a)
    r = B.bake_normals(*t, a.res, a.max_dist, count=True)
    nb, nt = r.test_counts()
    rays = r.ray_count()
    say(f"[gpu] axis-parallel rays: {nb / rays:.1f} box and {nt / rays:.2f} triangle tests per ray "
        f"({hF.shape[0]} triangles)")
    assert rays == 128 * 128
    assert nb / rays < 200 and nt / rays < 20  # ~8000 triangles: brute force would be thousands
    # every ray step is a lane of some whole-wave trip: a lane takes at most
    # one step per trip, and a wave makes a trip only while a lane steps
    trips = r.wave_trips()
    steps = nb // 2 + nt
    assert nb % 2 == 0
    assert steps <= 64 * trips
    assert trips <= steps
    for mode in (0, 1, 2):
        rm = B.bake_normals(*t, a.res, a.max_dist, count=True, trav_mode=mode)
        assert rm.test_counts() == (nb, nt)
        assert rm.wave_trips() <= steps <= 64 * rm.wave_trips()


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

def test_empty_low_poly_is_all_uncovered(B):
    a = make_config(1)
    t = list(B.to_device(a))
    t[4] = t[4][:0]
    t[5] = t[5][:0]
    r = B.bake_normals(*t, 64, 0.1)
    gm, gh = np_out(r)
    assert np.all(gh == -3) and np.allclose(gm, [0, 0, 1])
    assert r.ray_count() == 0


def test_empty_high_poly_is_all_miss(B):
    a = make_config(1)
    t = list(B.to_device(a))
    t[1] = t[1][:0]
    r = B.bake_normals(*t, a.res, a.max_dist)
    gm, gh = np_out(r)
    assert set(np.unique(gh).tolist()) == {-3, -1}
    assert np.allclose(gm[gh == -1], [0, 0, 1])


def test_single_triangle(B, oracle_lib):
    hV = np.float32([[-1, -1, 0.05], [3, -1, 0.05], [-1, 3, 0.05]])
    hF = np.int32([[0, 1, 2]])
    hN = np.tile(np.float32([0, 0, 1]), (3, 1))
    a = plane_asset(hV, hF, hN, res=16, lo_n=2, max_dist=0.1)
    r = run(B, a)
    check(oracle_lib, a, r)
    _, gh = np_out(r)
    assert np.all(gh == 0)


@pytest.mark.parametrize("res", [1, 2, 4])
def test_tiny_atlases(B, oracle_lib, res):
    a = make_config(1)
    a = Asset(a.name, a.hi_V, a.hi_F, a.hi_N, a.lo_V, a.lo_F, M.face_grid_atlas(80, res),
              res=res, max_dist=a.max_dist)
    r = run(B, a)
    check(oracle_lib, a, r)


def test_degenerate_lo_face_unreliable(B, oracle_lib):
    lV, lF = grid(2)
    F = lF.copy()
    F[3] = [F[3, 0], F[3, 0], F[3, 2]]
    uv = plane_uv(lV, lF)
    hV, hF, hN = _hi_plane(3, lambda x, y: 0.02 + 0 * x, (0, 0, 1))
    a = Asset("degen", hV, hF, hN, lV, F.astype(np.int32), uv, res=16, max_dist=0.1)
    r = run(B, a)
    check(oracle_lib, a, r)
    _, gh = np_out(r)
    assert (gh == -2).sum() > 0


def test_bad_indices_raise_status_not_fault(B):
    a = make_config(1)
    t = list(B.to_device(a))
    hF = t[1].clone()
    hF[5, 1] = 10 ** 8
    lF = t[4].clone()
    lF[3, 2] = -7
    r = B.bake_normals(t[0], hF, t[2], t[3], lF, t[5], a.res, a.max_dist)
    st = r.status()
    assert st & B.BAKE_STATUS_HI_INDEX and st & B.BAKE_STATUS_LO_INDEX


def test_rgb8_output(B, oracle_lib):
    a = make_config(1)
    r = run(B, a, rgb8=True)
    gm, _ = np_out(r)
    rgb = r.rgb8.cpu().numpy().reshape(-1, 3)
    exp = oracle_lib.rgb8(gm.astype(np.float64))
    # float32 vs float64 rounding of (x+1)*127.5+0.5 may differ by one code at
    # exact half steps
    assert np.abs(rgb.astype(int) - exp.astype(int)).max() <= 1
    assert (rgb != exp).mean() < 1e-3


# ---------------------------------------------------------------------------
# full-size workloads (sampled / BVH oracle)
# ---------------------------------------------------------------------------

def _full_size(B, oracle_lib, cfg, n_brute):
    a = make_config(cfg)
    r = run(B, a)
    gm, gh = np_out(r)
    say(f"[gpu] cfg{cfg}: GPU done, oracle BVH over all rays")
    ob = oracle_lib.bake(a, method="bvh")
    rep = compare(oracle_lib, a, ob, gm, gh)
    say(f"[gpu] cfg{cfg} full (oracle BVH):", rep)
    assert rep.ok(), str(rep)
    assert rep.n_covered == ob.texels.size  # the oracle's rasteriser decides coverage
    rp = compare_plain(oracle_lib, a, oracle_lib.bake(a, method="bvh", rule="plain", dilate_passes=0), gm, gh)
    say(f"[gpu] cfg{cfg} full (oracle BVH):", rp)
    assert rp.ok(), str(rp)
    # brute force on a seeded sample of covered texels
    rng = np.random.default_rng(cfg)
    sample = np.sort(rng.choice(ob.texels, size=n_brute, replace=False))
    obs = oracle_lib.bake(a, method="brute", texels=sample)
    rep2 = compare(oracle_lib, a, obs, gm, gh, check_dilation=False)
    say(f"[gpu] cfg{cfg} sample (brute force):", rep2)
    assert rep2.ok(), str(rep2)
    # the BVH oracle equals brute force on the sample
    pos = np.searchsorted(ob.texels, sample)
    assert np.array_equal(ob.hit[pos], obs.hit)
    return rep


def test_config2_full_size(B, oracle_lib):
    rep = _full_size(B, oracle_lib, 2, n_brute=256)
    assert rep.n_covered == 1082478


@pytest.mark.slow
def test_config3_full_size(B, oracle_lib):
    rep = _full_size(B, oracle_lib, 3, n_brute=64)
    assert rep.n_covered == 4328992
