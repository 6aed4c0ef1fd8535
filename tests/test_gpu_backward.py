"""GPU backward (through the C ABI) against the FP64 oracle adjoint.

The oracle differentiates the frozen-selection forward at the GPU's own hit
selection (the GPU's hit ids per texel; the texel -> face assignment and the
barycentrics are the rasteriser's exact integers, bit-identical on both
sides), with the same upstream gradient the GPU received.  Every entry of
dL/dlo_V and dL/dhi_N is compared, with no exclusions: relative L2 <= 1e-4
overall, and per entry |gpu - adjoint| <= 1e-3 |adjoint| + 1e-6 max|adjoint|
(+ for dL/dhi_N the FP32 noise term below).

The FP64 adjoint recomputes the hit weights beta of the selected triangle
exactly; the GPU's come from its FP32 forward, which moves them by up to the
comparator's weight noise bound (tests/compare.py, ``weight_slack``: the ray's
origin and direction rounding and the watertight test's arithmetic, divided by
the hit triangle's smallest altitude: ~1e-4 on the 1.3M-triangle noise
sphere, whose triangles are 3e-3 across at unit coordinates).  A hi_N term
beta_k h_bar with a small beta_k carries that absolute error, whatever the
backward's own arithmetic, so per entry of dL/dhi_N the tolerance adds the
oracle's first-order bound of how far its terms move under that perturbation
(oracle.c, orc_adjoint: bnoise / ghiN_sens).  The report also gives the
largest error in units of u = 2^-24 times the entry's summed term magnitudes
(the scale an FP32 evaluation of the sums is accurate to).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import compare as CMP  # noqa: E402
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


def _adjoint_at_gpu_selection(oracle_lib, a, r, gm):
    """The oracle's adjoint at the GPU's hit ids, fed the GPU's upstream
    gradient (float32 values widened exactly): (lo_V, hi_N, their term
    magnitudes, hi_N's weight-noise bound)."""
    g = gm.detach().cpu().numpy() if torch.is_tensor(gm) else np.asarray(gm, np.float32)
    hit = r.hit.cpu().numpy()
    return oracle_lib.adjoint_at(a, hit, g.astype(np.float64).reshape(-1, 3), magnitudes=True,
                                 bnoise=CMP.weight_noise(a, hit))


def test_backward_matches_oracle_adjoint_ripple(B, oracle_lib):
    a = make_config(1)
    rng = np.random.default_rng(3)
    gm = rng.normal(size=(a.res, a.res, 3)).astype(np.float32)
    r, t, gmt, glo, ghi = _run(B, a, gm)
    olo, ohi, mlo, mhi, shi = _adjoint_at_gpu_selection(oracle_lib, a, r, gmt)
    CMP.compare_grads("lo_V", glo, olo, mlo)
    CMP.compare_grads("hi_N", ghi, ohi, mhi, shi)
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


@pytest.mark.parametrize("n,off", [(12289, 0), (4097, 0), (3, 0), (8195, 1), (4096 * 5 + 2, 2)])
def test_sq_loss_ragged_and_unaligned(B, n, off):
    """Counts that are not a multiple of 4 or of the 4096-value block tile, and
    arrays that start off a 16-byte boundary (the 4-byte path)."""
    rng = np.random.default_rng(n)
    m = rng.normal(size=n + off).astype(np.float32)
    tg = rng.normal(size=n + off).astype(np.float32)
    loss, grad = B.sq_loss(torch.from_numpy(m).cuda()[off:], torch.from_numpy(tg).cuda()[off:])
    d = m[off:].astype(np.float64) - tg[off:]
    assert abs(float(loss.item()) - (d * d).sum()) <= 1e-5 * (d * d).sum()
    assert np.array_equal(grad.cpu().numpy(), (2.0 * (m[off:] - tg[off:])).astype(np.float32))


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
    [655,362 x 3] against the FP64 adjoint at the GPU's hit selection, every
    entry."""
    a = make_config(2, seed=0)
    say("[gpu] cfg4: oracle target from seed 1")
    tgt_asset = make_config(2, seed=1)
    tgt = oracle_lib.bake(tgt_asset, method="bvh", dilate_passes=0).map_raw
    r, t, gm_t, glo, ghi = _run(B, a, target=tgt)
    assert glo.shape == (10242, 3) and ghi.shape == (655362, 3)
    say("[gpu] cfg4: oracle adjoint at the GPU's selection")
    olo, ohi, mlo, mhi, shi = _adjoint_at_gpu_selection(oracle_lib, a, r, gm_t)
    CMP.compare_grads("lo_V", glo, olo, mlo)
    CMP.compare_grads("hi_N", ghi, ohi, mhi, shi)


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


def test_two_streams_equal_one_stream_bitwise(B):
    """The same asset with the low-poly work on a second stream (forward and
    backward) and with every stage on the caller's stream: the kernels and the
    sum orders are the same, so the outputs and gradients are equal bit for
    bit; a lost dependency between the streams would show here."""
    a = _large_asset(False)
    rng = np.random.default_rng(13)
    gm = torch.from_numpy(rng.normal(size=(a.res, a.res, 3)).astype(np.float32)).cuda()
    t = B.to_device(a)
    out = []
    for one in (False, True, False):
        say(f"[gpu] {a.name}: one_stream={one}")
        r = B.bake_normals(*t, a.res, a.max_dist, save=True, dilate_passes=2, one_stream=one)
        glo, ghi = B.bake_normals_backward(r, t, gm)
        torch.cuda.synchronize()
        out.append([x.clone() for x in (r.map, r.hit, glo, ghi)])
    for k in (1, 2):
        for x, y in zip(out[0], out[k]):
            assert torch.equal(x.view(torch.int32), y.view(torch.int32))
    assert np.abs(out[0][3].cpu().numpy()).sum() > 0


def test_backward_with_no_covered_texel_on_two_streams(B):
    a = _large_asset(True)
    gm = np.ones((a.res, a.res, 3))
    say(f"[gpu] {a.name}: backward with no rays")
    r, _, _, glo, ghi = _run(B, a, gm)
    assert r.ray_count() == 0
    assert not glo.any() and not ghi.any()


def test_non_finite_upstream_gradient_stays_in_its_vertices(B):
    """An infinite upstream gradient at one hit texel makes exactly the three
    vertices of its hit triangle NaN in dL/dhi_N; every other entry is bitwise
    what it is when that texel's gradient is 0 (each vertex sums only its own
    run of the sorted pairs)."""
    a = make_config(1)
    rng = np.random.default_rng(14)
    gm = rng.normal(size=(a.res, a.res, 3)).astype(np.float32)
    t = B.to_device(a)
    r = B.bake_normals(*t, a.res, a.max_dist, save=True, dilate_passes=0)
    hit = r.hit.cpu().numpy().reshape(-1)
    tex = int(np.nonzero(hit >= 0)[0][100])
    g0 = gm.copy().reshape(-1, 3)
    g0[tex] = 0.0
    ginf = gm.copy().reshape(-1, 3)
    ginf[tex] = [np.inf, 0.0, 0.0]
    out = []
    for g in (g0, ginf):
        _, ghi = B.bake_normals_backward(r, t, torch.from_numpy(g.reshape(a.res, a.res, 3)).cuda(), need_lo=False)
        torch.cuda.synchronize()
        out.append(ghi.cpu().numpy())
    tri = a.hi_F[hit[tex]]
    nan_rows = np.nonzero(np.isnan(out[1]).any(1))[0]
    assert set(nan_rows.tolist()) == set(int(v) for v in tri), (nan_rows, tri)
    keep = np.setdiff1d(np.arange(a.hi_V.shape[0]), tri)
    assert np.array_equal(out[0][keep].view(np.uint32), out[1][keep].view(np.uint32))
