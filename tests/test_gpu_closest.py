"""GPU closest-point query (the paper's own form of the correspondence step)
against the FP64 oracle, through the C ABI (tests/compare.py,
compare_closest, states the parity rules for this query)."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from compare import angle_deg, closest_near_ties, compare_closest  # noqa: E402
from planes import grid, plane_asset  # noqa: E402
from synth import Asset, make_config  # noqa: E402
from synth import meshes as M  # noqa: E402


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_26137_amd.bake as bake
    bake.lib()
    return bake


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(B, a, max_dist=None, **kw):
    t = B.to_device(a)
    md = a.max_dist if max_dist is None else max_dist
    r = B.bake_normals(*t, a.res, md, query="closest", **kw)
    torch.cuda.synchronize()
    assert r.status() == 0
    return r, r.map.cpu().numpy().reshape(-1, 3), r.hit.cpu().numpy().reshape(-1)


def bbox_diag(a):
    V = np.asarray(a.hi_V, np.float64)
    return float(np.linalg.norm(V.max(0) - V.min(0)))


@pytest.mark.parametrize("md", [0.1, None])
def test_ripple_closest_full(B, oracle_lib, md):
    a = make_config(1)
    if md is None:
        md = 0.01 * bbox_diag(a)  # the paper's filter: 1% of the bounding-box diagonal
    r, gm, gh = run(B, a, md)
    ob = oracle_lib.bake(a, kind="closest", max_dist=md)
    near = closest_near_ties(oracle_lib, a, ob)
    rep = compare_closest(oracle_lib, a, ob, gm, gh, near=near)
    say(f"[gpu] closest cfg1 md={md:.4f}: near ties {near.sum()}:", rep)
    assert rep.ok(), str(rep)
    assert rep.agree >= 1.0 - near.mean()
    assert (gh >= 0).sum() > 1000


@pytest.mark.parametrize("s,r,c", [(0.0, 0.0, 0.04), (0.3, -0.2, 0.01), (-0.25, 0.15, -0.08)])
def test_tilted_plane_closed_form(B, oracle_lib, s, r, c):
    n = 9
    V, F = grid(n, z=lambda x, y: s * x + r * y + c, x0=-0.25, y0=-0.25, size=1.5)
    N = np.stack([0.7 * V[:, 0], -0.4 * V[:, 1], np.ones(V.shape[0], np.float32)], 1).astype(np.float32)
    a = plane_asset(V, F, N, res=64, lo_n=8, max_dist=0.5)
    _, gm, gh = run(B, a, dilate_passes=0)
    ob = oracle_lib.bake(a, kind="closest")
    rep = compare_closest(oracle_lib, a, ob, gm, gh, check_dilation=False)
    say(f"[gpu] closest plane {s},{r},{c}:", rep)
    assert rep.ok(), str(rep)
    # closed form on tie-free texels: the projection onto the plane
    x, y = ob.P[:, 0], ob.P[:, 1]
    k = math.sqrt(1 + s * s + r * r)
    h = s * x + r * y + c
    qx, qy = x - s * h / (k * k), y - r * h / (k * k)
    hq = np.stack([0.7 * qx, -0.4 * qy, np.ones_like(qx)], 1)
    hq /= np.linalg.norm(hq, axis=1, keepdims=True)
    assert np.all(gh[ob.texels] >= 0)
    assert np.abs(gm[ob.texels] - hq).max() < 2e-4  # near-tie texels take a neighbour's edge point


def test_surface_onto_itself_is_z(B):
    V, F = M.icosphere(2)
    V = V.astype(np.float32)
    F = F.astype(np.int32)
    a = Asset("self", V, F, M.vertex_normals(V.astype(np.float64), F), V, F,
              M.face_grid_atlas(F.shape[0], 128), res=128, max_dist=0.01)
    _, gm, gh = run(B, a, dilate_passes=0)
    cov = gh != -3
    assert np.all(gh[cov] >= 0)
    z = np.zeros_like(gm[cov])
    z[:, 2] = 1.0
    ang = angle_deg(gm[cov], z)  # arctan2 form: arccos(z) is ill-conditioned at z ~ 1
    assert ang.max() < 1e-4


def test_sphere_and_holes_against_oracle(B, oracle_lib):
    """Noisy decimated sphere (holes: edge and vertex nearest points) at 256^2."""
    lV, lF = M.icosphere(2)
    hV, hF = M.icosphere(6)
    U = M.unit_directions(hV)
    hiV = M.displace(U, M.noise_radius(U, 9, 4, 0.03))
    hiV, hiF = M.decimate(hiV, hF, 30000, seed=9)
    hiF = hiF.astype(np.int32)
    a = Asset("holes", hiV, hiF, M.vertex_normals(hiV, hiF), lV.astype(np.float32),
              lF.astype(np.int32), M.face_grid_atlas(lF.shape[0], 256), res=256, max_dist=0.05)
    _, gm, gh = run(B, a)
    ob = oracle_lib.bake(a, kind="closest", method="bvh")
    rep = compare_closest(oracle_lib, a, ob, gm, gh)
    say("[gpu] closest holes:", rep)
    assert rep.ok(), str(rep)


def test_traversal_configs_identical(B):
    a = make_config(1)
    _, m0, h0 = run(B, a, 0.1)
    for blk in (64, 128, 256):
        for stk in (8, 16, 32):
            for mode in (0, 1, 2, 3):
                _, m, h = run(B, a, 0.1, trav_block=blk, trav_stack=stk, trav_mode=mode)
                assert np.array_equal(h, h0) and np.array_equal(m.view(np.uint32), m0.view(np.uint32))


def test_batch_closest_equals_single(B):
    assets = [make_config(1), make_config(1, seed=3)]
    singles = [run(B, a, 0.1) for a in assets]
    batch = B.BakeBatch([(*B.to_device(a), a.res, 0.1) for a in assets], query="closest")
    batch.forward()
    torch.cuda.synchronize()
    for i, (_, m, h) in enumerate(singles):
        assert np.array_equal(batch.hits[i].cpu().numpy().reshape(-1), h)
        assert np.array_equal(batch.maps[i].cpu().numpy().reshape(-1, 3).view(np.uint32), m.view(np.uint32))


def test_closest_rejects_save(B):
    a = make_config(1)
    t = B.to_device(a)
    with pytest.raises(B.BakeError) as e:
        B.bake_normals(*t, a.res, 0.1, query="closest", save=True)
    assert e.value.code == B.BAKE_E_UNSUPPORTED


def test_config2_closest_full_size(B, oracle_lib):
    """1.31M triangles onto the 20,480-triangle low-poly at 2048^2 with the
    paper's filter (1% of the bounding-box diagonal), against the FP64 BVH."""
    a = make_config(2)
    md = 0.01 * bbox_diag(a)
    r, gm, gh = run(B, a, md)
    say(f"[gpu] closest cfg2: GPU done (md {md:.4f}), oracle BVH")
    ob = oracle_lib.bake(a, kind="closest", method="bvh", max_dist=md)
    near = closest_near_ties(oracle_lib, a, ob)
    floor = 1.0 - near.mean()
    rep = compare_closest(oracle_lib, a, ob, gm, gh, near=near)
    say(f"[gpu] closest cfg2: near ties {near.sum()} ({near.mean():.4%}), agreement floor {floor:.6f}:", rep)
    assert rep.ok(), str(rep)
    assert rep.agree >= floor
