"""Batched bakes (bake_normals_batched / _backward) through the C ABI.

A batch runs every stage once over all assets; each asset must come out
bitwise equal to a single bake_normals / bake_normals_backward call on the same
inputs (which the other GPU tests check against the oracle), also when the
batch is recorded into a graph and replayed, and for every traversal
configuration the autotuner tries.  A sample of texels of a batched asset is
also checked directly against the oracle's brute force.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from synth import Asset, make_batch_assets, make_config  # noqa: E402
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


def _single_triangle_asset():
    hV = np.array([[-1, -1, 0.05], [1, -1, 0.05], [0, 1, 0.05]], np.float64)
    hF = np.array([[0, 1, 2]], np.int32)
    lV = np.array([[-1, -1, 0], [1, -1, 0], [0, 1, 0]], np.float32)
    lF = np.array([[0, 1, 2]], np.int32)
    uv = np.array([[[0.1, 0.1], [0.9, 0.1], [0.5, 0.9]]], np.float32)
    N = np.tile(np.array([[0.0, 0.0, 1.0]]), (3, 1))
    return Asset("tri", hV, hF, N, lV, lF, uv, res=32, max_dist=0.1)


def _empty_hi_asset():
    a = make_config(1)
    return Asset("nohi", a.hi_V[:3], np.zeros((0, 3), np.int32), a.hi_N[:3], a.lo_V, a.lo_F, a.lo_UV,
                 res=64, max_dist=0.1)


def _rayless_asset():
    """A low-poly triangle whose UV triangle covers no texel centre: no rays."""
    a = _single_triangle_asset()
    uv = np.array([[[0.501, 0.501], [0.503, 0.501], [0.501, 0.503]]], np.float32)
    return Asset("noray", a.hi_V, a.hi_F, a.hi_N, a.lo_V, a.lo_F, uv, res=32, max_dist=0.1)


def _mixed_assets():
    """Uneven small batch: generated assets of different sizes and atlases,
    the ripple sphere, a single triangle and an asset without high-poly."""
    gen = make_batch_assets(5, seed=7, hi_range=(2_000, 60_000), lo_range=(80, 2_000),
                            res_choices=(64, 128, 256), max_dist=0.1)
    return [gen[0], make_config(1), _single_triangle_asset(), gen[1], _empty_hi_asset(), gen[2],
            gen[3], gen[4]]


def _inputs(B, a):
    t = B.to_device(a)
    return (*t, a.res, a.max_dist)


def _bits(x):
    return x.contiguous().view(torch.int32).cpu().numpy()


def _single(B, a, dilate=2, save=False, grad_map=None, **kw):
    t = B.to_device(a)
    r = B.bake_normals(*t, a.res, a.max_dist, dilate_passes=dilate, save=save, rgb8=True, **kw)
    out = dict(map=_bits(r.map), hit=r.hit.cpu().numpy(), rgb8=r.rgb8.cpu().numpy(), rays=r.ray_count())
    if grad_map is not None:
        glo, ghi = B.bake_normals_backward(r, t, grad_map)
        out["glo"], out["ghi"] = _bits(glo), _bits(ghi)
    return out


def _check_batch_equals_single(B, batch, assets, singles, grads=False):
    rays = batch.ray_counts()
    for i, (a, s) in enumerate(zip(assets, singles)):
        assert rays[i] == s["rays"], (i, rays[i], s["rays"])
        assert np.array_equal(_bits(batch.maps[i]), s["map"]), f"asset {i} map"
        assert np.array_equal(batch.hits[i].cpu().numpy(), s["hit"]), f"asset {i} hit"
        if batch.rgb8[i] is not None:
            assert np.array_equal(batch.rgb8[i].cpu().numpy(), s["rgb8"]), f"asset {i} rgb8"
        if grads:
            assert np.array_equal(_bits(batch.grad_lo_V[i]), s["glo"]), f"asset {i} grad lo_V"
            assert np.array_equal(_bits(batch.grad_hi_N[i]), s["ghi"]), f"asset {i} grad hi_N"


def test_batch_forward_equals_single_bakes(B):
    assets = _mixed_assets()
    say("[gpu] batch fwd: sizes", [(a.hi_F.shape[0], a.lo_F.shape[0], a.res) for a in assets])
    singles = [_single(B, a) for a in assets]
    batch = B.BakeBatch([_inputs(B, a) for a in assets], rgb8=True)
    batch.forward()
    torch.cuda.synchronize()
    assert batch.status() == 0
    _check_batch_equals_single(B, batch, assets, singles)
    # texels were really traced (generated assets are randomly decimated, so
    # their high-poly has holes and a good part of the rays miss)
    for i in (0, 1, 3):
        h = batch.hits[i].cpu().numpy()
        assert (h >= 0).sum() > 0.3 * (h != B.BAKE_UNCOVERED).sum(), i


def test_batch_backward_equals_single(B):
    assets = _mixed_assets()
    rng = np.random.default_rng(11)
    gms = [torch.from_numpy(rng.normal(size=(a.res, a.res, 3)).astype(np.float32)).cuda() for a in assets]
    singles = [_single(B, a, dilate=0, save=True, grad_map=g) for a, g in zip(assets, gms)]
    batch = B.BakeBatch([_inputs(B, a) for a in assets], save=True, dilate_passes=0, rgb8=True)
    for i, g in enumerate(gms):
        batch.grad_maps[i].copy_(g)
    batch.forward()
    batch.backward()
    torch.cuda.synchronize()
    _check_batch_equals_single(B, batch, assets, singles, grads=True)
    assert any(np.abs(s["glo"]).sum() > 0 for s in singles)


def test_batch_backward_with_rayless_assets(B):
    """Assets without a single ray before, between and after assets with rays:
    the per-asset prefix of the backward sort's tiles has empty ranges, and
    the sort's grid (sized for every asset's capacity) is mostly idle blocks.
    Forward and backward equal the single bakes bit for bit."""
    gen = make_batch_assets(3, seed=13, hi_range=(2_000, 30_000), lo_range=(80, 800),
                            res_choices=(64, 128), max_dist=0.1)
    assets = [_rayless_asset(), gen[0], _rayless_asset(), _rayless_asset(), gen[1], _rayless_asset(), gen[2],
              _rayless_asset()]
    rng = np.random.default_rng(12)
    gms = [torch.from_numpy(rng.normal(size=(a.res, a.res, 3)).astype(np.float32)).cuda() for a in assets]
    singles = [_single(B, a, dilate=0, save=True, grad_map=g) for a, g in zip(assets, gms)]
    assert [s["rays"] == 0 for s in singles] == [a.name == "noray" for a in assets]
    batch = B.BakeBatch([_inputs(B, a) for a in assets], save=True, dilate_passes=0, rgb8=True)
    for i, g in enumerate(gms):
        batch.grad_maps[i].copy_(g)
    batch.forward()
    batch.backward()
    torch.cuda.synchronize()
    assert batch.status() == 0
    _check_batch_equals_single(B, batch, assets, singles, grads=True)
    for a, s in zip(assets, singles):
        if a.name == "noray":
            assert not np.any(s["glo"]) and not np.any(s["ghi"])
        else:
            assert np.abs(s["glo"]).sum() > 0


def test_batch_order_does_not_matter(B):
    assets = _mixed_assets()
    perm = [5, 2, 7, 0, 4, 1, 6, 3]
    b1 = B.BakeBatch([_inputs(B, a) for a in assets])
    b2 = B.BakeBatch([_inputs(B, assets[p]) for p in perm])
    b1.forward()
    b2.forward()
    torch.cuda.synchronize()
    for j, p in enumerate(perm):
        assert np.array_equal(_bits(b2.maps[j]), _bits(b1.maps[p]))
        assert torch.equal(b2.hits[j], b1.hits[p])


def test_batch_graph_replay(B):
    """Forward + backward recorded into one graph: every replay, with eager
    work and synchronisations between replays, equals the eager results."""
    assets = _mixed_assets()[:5]
    rng = np.random.default_rng(12)
    batch = B.BakeBatch([_inputs(B, a) for a in assets], save=True, dilate_passes=2)
    for g in batch.grad_maps:
        g.copy_(torch.from_numpy(rng.normal(size=tuple(g.shape)).astype(np.float32)))
    batch.forward()
    batch.backward()
    torch.cuda.synchronize()
    ref = [(_bits(m), h.cpu().numpy(), _bits(gl), _bits(gh))
           for m, h, gl, gh in zip(batch.maps, batch.hits, batch.grad_lo_V, batch.grad_hi_N)]
    graph = batch.capture()
    for rep in range(3):
        for m, h, gl, gh in zip(batch.maps, batch.hits, batch.grad_lo_V, batch.grad_hi_N):
            m.fill_(7.0)
            h.fill_(-9)
            gl.fill_(3.0)
            gh.fill_(3.0)
        x = torch.randn(1 << 20, device="cuda")
        torch.cuda.synchronize()
        graph.replay()
        y = (x * 2).sum()
        torch.cuda.synchronize()
        assert torch.isfinite(y)
        for i, (m, h, gl, gh) in enumerate(zip(batch.maps, batch.hits, batch.grad_lo_V, batch.grad_hi_N)):
            assert np.array_equal(_bits(m), ref[i][0]), (rep, i)
            assert np.array_equal(h.cpu().numpy(), ref[i][1]), (rep, i)
            assert np.array_equal(_bits(gl), ref[i][2]), (rep, i)
            assert np.array_equal(_bits(gh), ref[i][3]), (rep, i)


def test_autotune_every_config_same_result(B, tmp_path):
    assets = _mixed_assets()[:4]
    batch = B.BakeBatch([_inputs(B, a) for a in assets])
    batch.forward()
    torch.cuda.synchronize()
    ref = [(_bits(m), h.cpu().numpy()) for m, h in zip(batch.maps, batch.hits)]
    cache = str(tmp_path / "tune.json")
    out = B.autotune(batch, reps=1, cache_path=cache)
    say("[gpu] autotune", out["block"], out["stack"], out["mode"])
    assert (out["block"], out["stack"], out["mode"]) in B.TRAV_CONFIGS
    assert len(out["ms"]) == 36 and all(v > 0 for v in out["ms"].values())
    # every configuration gives the same results (the last one tried stays)
    for i, (m, h) in enumerate(zip(batch.maps, batch.hits)):
        assert np.array_equal(_bits(m), ref[i][0]) and np.array_equal(h.cpu().numpy(), ref[i][1])
    b2 = B.BakeBatch([_inputs(B, a) for a in assets])
    assert B.apply_tuning(b2, cache)
    assert (b2.opts.trav_block, b2.opts.trav_stack, b2.opts.trav_mode) == \
        (out["block"], out["stack"], out["mode"])


def test_batch_errors(B):
    a = make_config(1)
    batch = B.BakeBatch([_inputs(B, a)])
    with pytest.raises(B.BakeError) as e:  # made without save
        batch.backward()
    assert e.value.code == B.BAKE_E_STATE


def test_backward_on_overwritten_workspace_writes_nothing(B):
    """The forward seals its saved state with a nonce; a backward that finds
    another value (the workspace was overwritten) writes nothing and raises
    BAKE_STATUS_STATE."""
    a = make_config(1)
    batch = B.BakeBatch([_inputs(B, a)], save=True, dilate_passes=0)
    batch.grad_maps[0].normal_()
    batch.forward()
    batch.grad_lo_V[0].fill_(5.0)
    batch.grad_hi_N[0].fill_(5.0)
    # batch counters follow the 256-byte status block and the per-asset
    # counters (16 words per asset, padded to 256 bytes); the nonce is word 1
    seal = 256 + 256 + 4
    batch.workspace[seal:seal + 4].zero_()
    batch.backward()
    torch.cuda.synchronize()
    assert torch.all(batch.grad_lo_V[0] == 5.0) and torch.all(batch.grad_hi_N[0] == 5.0)
    assert batch.status() & B.BAKE_STATUS_STATE
    # a fresh forward re-seals: the backward runs again
    batch.forward()
    batch.backward()
    torch.cuda.synchronize()
    assert not torch.all(batch.grad_lo_V[0] == 5.0)
    assert batch.status() == 0


def _sample(oracle_lib, a, n, seed):
    face, _ = oracle_lib.raster(a.lo_UV, a.res)
    cov = np.nonzero(face >= 0)[0]
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(cov, size=min(n, cov.size), replace=False))


# a sample of n texels cannot measure a 0.1 % disagreement rate; instead the
# number of (verified) ties in it is bounded: at a true rate of 0.1 %, more
# than 3 ties in 500 texels has probability < 2e-3
MAX_TIES_PER_500 = 3


def test_batched_asset_sample_against_oracle(B, oracle_lib):
    """500 seeded texels of each of three generated batch assets against the
    oracle's brute force (independent of the single-bake path)."""
    from compare import compare, compare_plain
    assets = make_batch_assets(3, seed=3, hi_range=(20_000, 80_000), lo_range=(500, 3_000),
                               res_choices=(256,), max_dist=0.1)
    batch = B.BakeBatch([_inputs(B, a) for a in assets], dilate_passes=0)
    batch.forward()
    torch.cuda.synchronize()
    for i, a in enumerate(assets):
        sample = _sample(oracle_lib, a, 500, 100 + i)
        gm, gh = batch.maps[i].cpu().numpy(), batch.hits[i].cpu().numpy()
        ob = oracle_lib.bake(a, method="brute", texels=sample, dilate_passes=0)
        rep = compare(oracle_lib, a, ob, gm, gh, check_dilation=False, agree_min=None)
        say(f"[gpu] batch asset {i} sample (brute force):", rep)
        assert rep.ok(), str(rep)
        assert rep.n_disagree <= MAX_TIES_PER_500
        obp = oracle_lib.bake(a, method="brute", texels=sample, dilate_passes=0, rule="plain")
        rp = compare_plain(oracle_lib, a, obp, gm, gh)
        say(f"[gpu] batch asset {i} sample:", rp)
        assert rp.ok(), str(rp)


@pytest.mark.slow
def test_batch_workload_against_oracle(B, oracle_lib):
    """The 64-asset batch the benchmark times (24.7M high-poly triangles in
    all, 53k-1.87M per asset, atlases 512-2048, holes from the decimation),
    forward + backward in one batched call: 500 seeded covered texels of
    every asset against the oracle's brute force (robust rule, plain-rule
    ties), and the backward of four assets (the smallest, the largest and two
    seeded picks) against the FP64 adjoint at the GPU's hit selection."""
    from compare import compare, compare_grads, compare_plain, weight_noise
    say("[gpu] batch workload: generating 64 assets")
    assets = make_batch_assets(64, seed=0, workers=8)
    batch = B.BakeBatch([_inputs(B, a) for a in assets], save=True, dilate_passes=0)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(31)
    for g in batch.grad_maps:
        g.normal_(generator=gen)
    say("[gpu] batch workload: forward + backward")
    batch.forward()
    batch.backward()
    torch.cuda.synchronize()
    assert batch.status() == 0
    n_all = n_dis = 0
    for i, a in enumerate(assets):
        sample = _sample(oracle_lib, a, 500, 1000 + i)
        gm, gh = batch.maps[i].cpu().numpy(), batch.hits[i].cpu().numpy()
        ob = oracle_lib.bake(a, method="brute", texels=sample, dilate_passes=0)
        rep = compare(oracle_lib, a, ob, gm, gh, check_dilation=False, agree_min=None)
        obp = oracle_lib.bake(a, method="brute", texels=sample, dilate_passes=0, rule="plain")
        rp = compare_plain(oracle_lib, a, obp, gm, gh)
        say(f"[gpu] batch asset {i} ({a.hi_F.shape[0]} tris, {a.res}^2): {rep} | {rp}")
        assert rep.ok(), (i, str(rep))
        assert rp.ok(), (i, str(rp))
        assert rep.n_disagree <= MAX_TIES_PER_500, i
        n_all += rep.n_compared
        n_dis += rep.n_disagree
    say(f"[gpu] batch workload: {n_all} sampled texels, {n_dis} verified ties, "
        f"agreement {1 - n_dis / n_all:.6f}")
    assert 1 - n_dis / n_all >= 0.999
    sizes = np.array([a.hi_F.shape[0] for a in assets])
    rng = np.random.default_rng(5)
    picks = [int(sizes.argmin()), int(sizes.argmax())]
    picks += [int(x) for x in rng.choice([k for k in range(64) if k not in picks], 2, replace=False)]
    for i in picks:
        a = assets[i]
        hit = batch.hits[i].cpu().numpy()
        olo, ohi, mlo, mhi, shi = oracle_lib.adjoint_at(
            a, hit, batch.grad_maps[i].cpu().numpy().astype(np.float64).reshape(-1, 3), magnitudes=True,
            bnoise=weight_noise(a, hit))
        say(f"[gpu] batch asset {i} ({a.hi_F.shape[0]} tris):")
        compare_grads("lo_V", batch.grad_lo_V[i].cpu().numpy(), olo, mlo, say=say)
        compare_grads("hi_N", batch.grad_hi_N[i].cpu().numpy(), ohi, mhi, shi, say=say)
