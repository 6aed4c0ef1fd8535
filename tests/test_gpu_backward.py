"""GPU backward (through the C ABI) against the FP64 oracle adjoint.

The oracle differentiates its own bake (its own hit selection); the GPU
differentiates its bake.  Where the two picked different triangles at a tie
the per-ray terms differ legitimately, so per-entry checks skip the vertices
such texels touch; the overall relative L2 error covers everything.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

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


def _excluded(asset, ob, gpu_hit):
    """Low-poly vertices (2-ring) and high-poly vertices touched by texels whose
    hit id differs between the GPU and the oracle."""
    tex = ob.texels
    dis = tex[gpu_hit.reshape(-1)[tex] != ob.status[tex]]
    lo_ex = np.zeros(asset.lo_V.shape[0], bool)
    hi_ex = np.zeros(asset.hi_V.shape[0], bool)
    if dis.size:
        faces = ob.face[dis]
        v1 = np.unique(asset.lo_F[faces])
        ring = np.isin(asset.lo_F, v1).any(1)
        v2 = np.unique(asset.lo_F[ring])
        ring2 = np.isin(asset.lo_F, v2).any(1)
        lo_ex[np.unique(asset.lo_F[ring2])] = True
        for ids in (gpu_hit.reshape(-1)[dis], ob.status[dis]):
            ids = ids[ids >= 0]
            hi_ex[np.unique(asset.hi_F[ids])] = True
    return lo_ex, hi_ex


def _compare_grads(name, g_gpu, g_orc, excl):
    g_gpu = np.asarray(g_gpu, np.float64)
    rel_all = np.linalg.norm(g_gpu - g_orc) / max(np.linalg.norm(g_orc), 1e-30)
    keep = ~excl
    rel_l2 = np.linalg.norm(g_gpu[keep] - g_orc[keep]) / max(np.linalg.norm(g_orc[keep]), 1e-30)
    err = np.abs(g_gpu[keep] - g_orc[keep])
    # an entry sums the contributions of many rays; the FP32 error of such a
    # sum is relative to the sum of the contributions' magnitudes, which can
    # be far larger than the result when they cancel: hence an absolute floor
    # of 1e-5 of the largest entry next to the 1e-3 relative bound
    tol = 1e-3 * np.abs(g_orc[keep]) + 1e-5 * np.abs(g_orc).max()
    worst = float((err / np.maximum(tol, 1e-300)).max()) if err.size else 0.0
    say(f"[gpu] grad {name}: rel L2 {rel_l2:.2e} (all entries {rel_all:.2e}), excluded "
        f"{int(excl.sum())}, worst err/tol {worst:.3f}")
    assert rel_l2 <= 1e-4, rel_l2
    assert np.all(err <= tol)
    return rel_l2


def _run(B, a, grad_map_np=None, target=None):
    t = B.to_device(a)
    r = B.bake_normals(*t, a.res, a.max_dist, save=True, dilate_passes=0)
    if target is not None:
        _, gm = B.sq_loss(r.map, torch.from_numpy(target.reshape(a.res, a.res, 3).astype(np.float32)).cuda())
    else:
        gm = torch.from_numpy(grad_map_np.astype(np.float32)).cuda()
    glo, ghi = B.bake_normals_backward(r, t, gm)
    torch.cuda.synchronize()
    return r, t, gm, glo.cpu().numpy(), ghi.cpu().numpy()


def test_backward_matches_oracle_adjoint_ripple(B, oracle_lib):
    a = make_config(1)
    rng = np.random.default_rng(3)
    gm = rng.normal(size=(a.res, a.res, 3))
    r, t, _, glo, ghi = _run(B, a, gm)
    ob = oracle_lib.bake(a)
    olo, ohi = oracle_lib.bake_adjoint(a, ob, gm.reshape(-1, 3))
    lo_ex, hi_ex = _excluded(a, ob, r.hit.cpu().numpy())
    _compare_grads("lo_V", glo, olo, np.repeat(lo_ex[:, None], 3, 1))
    _compare_grads("hi_N", ghi, ohi, np.repeat(hi_ex[:, None], 3, 1))
    assert np.abs(ohi).sum() > 0 and np.abs(olo).sum() > 0


def test_backward_bitwise_repeatable(B):
    a = make_config(1)
    rng = np.random.default_rng(5)
    gm = rng.normal(size=(a.res, a.res, 3))
    _, _, _, glo1, ghi1 = _run(B, a, gm)
    for _ in range(2):
        _, _, _, glo2, ghi2 = _run(B, a, gm)
        assert np.array_equal(glo1.view(np.uint32), glo2.view(np.uint32))
        assert np.array_equal(ghi1.view(np.uint32), ghi2.view(np.uint32))


def test_backward_ignores_non_hit_texels(B):
    a = make_config(1)
    rng = np.random.default_rng(6)
    gm = rng.normal(size=(a.res, a.res, 3))
    r, t, _, glo, ghi = _run(B, a, gm)
    hit = r.hit.cpu().numpy()
    gm2 = gm.copy()
    gm2[hit < 0] = 1e6
    _, _, _, glo2, ghi2 = _run(B, a, gm2)
    assert np.array_equal(glo, glo2) and np.array_equal(ghi, ghi2)


def test_backward_without_saved_forward_is_an_error(B):
    a = make_config(1)
    t = B.to_device(a)
    r = B.bake_normals(*t, a.res, a.max_dist, save=True, dilate_passes=0)
    # a later forward without save on the same workspace drops the saved state
    B.bake_normals(*t, a.res, a.max_dist, dilate_passes=0, workspace=r.workspace)
    with pytest.raises(B.BakeError) as e:
        B.bake_normals_backward(r, t, torch.zeros((a.res, a.res, 3), device="cuda"))
    assert e.value.code == B.BAKE_E_STATE


def test_sq_loss(B):
    rng = np.random.default_rng(8)
    m = rng.normal(size=(64, 64, 3)).astype(np.float32)
    tg = rng.normal(size=(64, 64, 3)).astype(np.float32)
    loss, grad = B.sq_loss(torch.from_numpy(m).cuda(), torch.from_numpy(tg).cuda())
    d = m.astype(np.float64) - tg
    assert abs(float(loss.item()) - (d * d).sum()) <= 1e-5 * (d * d).sum()
    assert np.array_equal(grad.cpu().numpy(), (2.0 * (m - tg)).astype(np.float32))


def test_autograd_function(B):
    a = make_config(1)
    hi_V, hi_F, hi_N, lo_V, lo_F, lo_UV = B.to_device(a)
    lo_V = lo_V.clone().requires_grad_(True)
    hi_N = hi_N.clone().requires_grad_(True)
    target = torch.zeros((a.res, a.res, 3), device="cuda")
    target[..., 2] = 1.0
    m, hit = B.BakeNormals.apply(lo_V, hi_N, hi_V, hi_F, lo_F, lo_UV, a.res, a.max_dist)
    loss = ((m - target) ** 2).sum()
    loss.backward()
    # the same through the explicit calls
    t = (hi_V, hi_F, hi_N.detach(), lo_V.detach(), lo_F, lo_UV)
    r = B.bake_normals(*t, a.res, a.max_dist, save=True, dilate_passes=0)
    _, gm = B.sq_loss(r.map, target)
    glo, ghi = B.bake_normals_backward(r, t, gm)
    assert torch.equal(lo_V.grad, glo) and torch.equal(hi_N.grad, ghi)
    assert not hit.requires_grad


def test_differentiation_workload_full_size(B, oracle_lib):
    """1.31M-triangle high-poly onto the 20,480-triangle low-poly at 2048^2:
    loss = sum of squared differences to the map baked (by the oracle) from a
    second noise seed; gradients w.r.t. lo_V [10,242 x 3] and hi_N
    [655,362 x 3] against the FP64 adjoint."""
    a = make_config(2, seed=0)
    say("[gpu] cfg4: oracle target from seed 1")
    tgt_asset = make_config(2, seed=1)
    tgt = oracle_lib.bake(tgt_asset, method="bvh", dilate_passes=0).map_raw
    r, t, gm_t, glo, ghi = _run(B, a, target=tgt)
    assert glo.shape == (10242, 3) and ghi.shape == (655362, 3)
    say("[gpu] cfg4: oracle bake + adjoint")
    ob = oracle_lib.bake(a, method="bvh", dilate_passes=0)
    go = 2.0 * (ob.map_raw - tgt)
    olo, ohi = oracle_lib.bake_adjoint(a, ob, go)
    lo_ex, hi_ex = _excluded(a, ob, r.hit.cpu().numpy())
    _compare_grads("lo_V", glo, olo, np.repeat(lo_ex[:, None], 3, 1))
    _compare_grads("hi_N", ghi, ohi, np.repeat(hi_ex[:, None], 3, 1))


def _large_asset(uv_zero, seed=9):
    # 81,920 high-poly faces: enough for the backward to run its low-poly
    # chain on the second stream, forked after the sort's first histogram
    lV, lF = M.icosphere(2)
    hV, hF = M.icosphere(6)
    U = M.unit_directions(hV)
    hiV = M.displace(U, M.noise_radius(U, seed, 4, 0.03))
    hiF = hF.astype(np.int32)
    res = 256
    uv = M.face_grid_atlas(lF.shape[0], res)
    if uv_zero:
        uv = np.zeros_like(uv)  # every chart collapsed to a point: no texel covered
    return Asset("noise_L6_L2_256" + ("_nouv" if uv_zero else ""), hiV, hiF, M.vertex_normals(hiV, hiF),
                 lV.astype(np.float32), lF.astype(np.int32), uv, res=res, max_dist=0.12)


def test_backward_on_two_streams_is_repeatable(B):
    a = _large_asset(False)
    assert a.hi_F.shape[0] >= 65536
    rng = np.random.default_rng(12)
    gm = rng.normal(size=(a.res, a.res, 3))
    say(f"[gpu] {a.name}: backward twice")
    r, _, _, glo1, ghi1 = _run(B, a, gm)
    assert r.ray_count() > 0 and np.abs(ghi1).sum() > 0 and np.abs(glo1).sum() > 0
    _, _, _, glo2, ghi2 = _run(B, a, gm)
    assert np.array_equal(glo1.view(np.uint32), glo2.view(np.uint32))
    assert np.array_equal(ghi1.view(np.uint32), ghi2.view(np.uint32))


def test_backward_with_no_covered_texel_on_two_streams(B):
    a = _large_asset(True)
    gm = np.ones((a.res, a.res, 3))
    say(f"[gpu] {a.name}: backward with no rays")
    r, _, _, glo, ghi = _run(B, a, gm)
    assert r.ray_count() == 0
    assert not glo.any() and not ghi.any()
