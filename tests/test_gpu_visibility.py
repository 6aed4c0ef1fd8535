"""GPU hidden-face removal (Sec. 6.2) against the FP64 oracle, through the C
ABI: every camera ray's first hit (ids agree on 99.9 % of the rays, and every
disagreement is explained by the FP32 noise at the hit rule's fences: see
compare.check_first_hits), the visibility mask (every face seen by one side
only is named by such a ray), and the flood fill (bit-exact: the oracle's fill
from the GPU's visible faces)."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from compare import check_first_hits  # noqa: E402
from planes import grid, grid_cell_triangle  # noqa: E402
from synth import meshes as M  # noqa: E402

TAN30 = math.tan(math.radians(30.0))


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


def run(B, V, F, eyes, target, tan_half, res, t_far, **kw):
    say(f"[gpu] visibility n_f={F.shape[0]} views={eyes.shape[0]} res={res} {kw}")
    d = torch.device("cuda")
    r = B.visibility(torch.from_numpy(np.ascontiguousarray(V, np.float32)).to(d),
                     torch.from_numpy(np.ascontiguousarray(F, np.int32)).to(d),
                     torch.from_numpy(np.ascontiguousarray(eyes, np.float32)).to(d), target, tan_half, res,
                     t_far, **kw)
    torch.cuda.synchronize()
    return r


def check_rays(oracle_lib, V, F, P, D, g_ids, o_ids, o_t, t_far, min_agree=0.999):
    """Per-ray parity (compare.check_first_hits states the rule); returns the
    faces that disagreeing rays name (either side)."""
    method = "brute" if F.shape[0] <= 200_000 else "bvh"
    rep = check_first_hits(oracle_lib, V, F, P, D, g_ids, o_ids, o_t, t_far, min_agree, method)
    say("[gpu]", rep)
    assert rep.ok(), str(rep)
    return rep.tie_faces


def check_masks(oracle_lib, V, F, r, o_vis, tie_faces):
    g_vis = r.visible.cpu().numpy()
    diff = np.nonzero(g_vis != o_vis)[0]
    assert set(diff.tolist()) <= tie_faces
    g_ext = r.exterior.cpu().numpy()
    assert np.array_equal(g_ext, oracle_lib.flood_fill(V, F, g_vis))
    assert np.all(g_ext >= g_vis)
    return g_vis, g_ext


def test_nested_spheres_against_brute_force(B, oracle_lib):
    V, F, n_out = M.hidden_face_mesh(outer_level=3, inner_level=2)
    eyes = M.sphere_viewpoints(16, [0, 0, 0], 2.5)
    res, t_far = 64, 5.0
    r = run(B, V, F, eyes, [0, 0, 0], TAN30, res, t_far, first_hit=True)
    assert r.status() == 0
    P, D = oracle_lib.camera_rays(eyes, [0, 0, 0], TAN30, res)
    o_ids, o_t = oracle_lib.first_hit(V, F, P, D, t_far, "brute")
    ties = check_rays(oracle_lib, V, F, P, D, r.first_hit.cpu().numpy(), o_ids, o_t, t_far)
    o_vis = np.zeros(F.shape[0], bool)
    o_vis[o_ids[o_ids >= 0]] = True
    g_vis, g_ext = check_masks(oracle_lib, V, F, r, o_vis, ties)
    assert not g_vis[n_out:].any() and not g_ext[n_out:].any()  # the inner sphere stays hidden
    assert g_ext[:n_out].all()                                    # the fill closes the shell


def test_plane_closed_form(B):
    n = 16
    V, F = grid(n)
    eye = np.array([[0.43, 0.61, 1.7]], np.float32)
    res = 64
    tan_half = math.tan(math.radians(12))
    target = [float(eye[0, 0]), float(eye[0, 1]), 0.0]
    r = run(B, V, F, eye, target, tan_half, res, 10.0, first_hit=True)
    ids = r.first_hit.cpu().numpy().reshape(-1)
    # the FP32 ray of pixel (i, j): plane point e + t d with t = -e_z / d_z
    c = (2 * (np.arange(res) + 0.5) / res - 1) * tan_half
    # forward -z, helper x: right (0,-1,0), up (1,0,0): x along -y, y along +x
    X, Y = np.meshgrid(c, -c)
    qx = eye[0, 0] + Y * eye[0, 2]
    qy = eye[0, 1] - X * eye[0, 2]
    fx, fy = (qx * n) % 1, (qy * n) % 1
    clear = (np.minimum.reduce([fx, 1 - fx, fy, 1 - fy, np.abs(fx - fy)]) > 1e-4).reshape(-1)
    expected = grid_cell_triangle(qx.reshape(-1), qy.reshape(-1), n)
    assert clear.mean() > 0.9
    assert np.array_equal(ids[clear], expected[clear])


def test_occluded_plane(B):
    n = 6
    V1, F1 = grid(n, z=lambda x, y: 0.0 * x)
    V2, F2 = grid(n, z=lambda x, y: 0.0 * x - 0.5)
    V = np.concatenate([V1, V2])
    F = np.concatenate([F1, F2 + V1.shape[0]]).astype(np.int32)
    nf = F1.shape[0]
    for z, front in ((2.0, 0), (-2.5, 1)):
        r = run(B, V, F, np.array([[0.5, 0.5, z]], np.float32), [0.5, 0.5, -0.25], math.tan(math.radians(8)),
                32, 10.0)
        vis = r.visible.cpu().numpy()
        assert vis[front * nf:(front + 1) * nf].any() and not vis[(1 - front) * nf:(2 - front) * nf].any()


def test_fill_stops_at_flipped_band(B, oracle_lib):
    """Few views leave the back of a sphere unseen; the fill closes it except
    where a band of faces is wound the other way: those join only if seen."""
    V, F = M.icosphere(3)
    V = V.astype(np.float32)
    F = F.astype(np.int32).copy()
    c = V[F].mean(1)
    band = np.abs(c[:, 2] + 0.3) < 0.08
    F[band] = F[band][:, ::-1]
    eyes = np.array([[0, 0, 3.0], [0.3, 0.2, 2.8]], np.float32)
    r = run(B, V, F, eyes, [0, 0, 0], TAN30, 96, 6.0, first_hit=True)
    P, D = oracle_lib.camera_rays(eyes, [0, 0, 0], TAN30, 96)
    o_ids, o_t = oracle_lib.first_hit(V, F, P, D, 6.0, "bvh")
    ties = check_rays(oracle_lib, V, F, P, D, r.first_hit.cpu().numpy(), o_ids, o_t, 6.0)
    o_vis = np.zeros(F.shape[0], bool)
    o_vis[o_ids[o_ids >= 0]] = True
    g_vis, g_ext = check_masks(oracle_lib, V, F, r, o_vis, ties)
    assert not g_vis[c[:, 2] < -0.5].any()           # the far cap is not seen
    assert not g_ext[band & ~g_vis].any()            # unseen flipped faces never join
    assert not g_ext[c[:, 2] < -0.45].any()          # the band cuts the far cap off
    assert g_ext[(c[:, 2] > -0.2) & ~band].all()     # the near side closes


def test_repeat_bitwise_and_counters(B):
    V, F, _ = M.hidden_face_mesh(outer_level=3, inner_level=2)
    eyes = M.sphere_viewpoints(8, [0, 0, 0], 2.5)
    r1 = run(B, V, F, eyes, [0, 0, 0], TAN30, 48, 5.0, first_hit=True)
    r2 = run(B, V, F, eyes, [0, 0, 0], TAN30, 48, 5.0, first_hit=True, count=True)
    assert torch.equal(r1.first_hit, r2.first_hit) and torch.equal(r1.exterior, r2.exterior)
    nb, nt, trips = r2.counter(1), r2.counter(2), r2.counter(3)
    rays = 8 * 48 * 48
    assert nb > 2 * rays and nt >= (r2.first_hit >= 0).sum().item()
    assert nb % 2 == 0 and trips <= nb // 2 + nt <= 64 * trips


def test_empty_single_and_bad_index(B):
    eyes = np.array([[0, 0, 2.0]], np.float32)
    r = run(B, np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), eyes, [0, 0, 0], TAN30, 16, 5.0,
            first_hit=True)
    assert r.status() == 0 and (r.first_hit.cpu().numpy() == -1).all() and r.visible.numel() == 0
    V = np.array([[-1, -1, 0], [1, -1, 0], [0, 1, 0]], np.float32)
    F = np.array([[0, 1, 2]], np.int32)
    r = run(B, V, F, eyes, [0, 0, 0], TAN30, 16, 5.0, first_hit=True)
    assert r.visible.cpu().numpy().tolist() == [True] and r.exterior.cpu().numpy().tolist() == [True]
    assert (r.first_hit.cpu().numpy() >= 0).sum() > 20
    F2 = np.array([[0, 1, 2], [0, 1, 7]], np.int32)
    r = run(B, V, F2, eyes, [0, 0, 0], TAN30, 16, 5.0)
    assert r.status() & B.BAKE_STATUS_HI_INDEX
    assert r.visible.cpu().numpy().tolist() == [True, False]
    assert r.exterior.cpu().numpy().tolist() == [True, False]


def test_paper_configuration_sampled(B, oracle_lib):
    """512 viewpoints x 1024^2 rays on the 21,760-face nested mesh (the
    paper's settings and mesh size): the inner sphere is never seen, the fill
    is the oracle's from the GPU's visible faces, and a seeded sample of rays
    matches the FP64 BVH one by one."""
    V, F, n_out = M.hidden_face_mesh()
    eyes = M.sphere_viewpoints(512, [0, 0, 0], 2.5)
    res, t_far = 1024, 5.0
    r = run(B, V, F, eyes, [0, 0, 0], TAN30, res, t_far, first_hit=True)
    assert r.status() == 0
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(512 * res * res, size=20000, replace=False))
    g_ids = r.first_hit.view(-1)[torch.from_numpy(sample).cuda()].cpu().numpy()
    P, D = oracle_lib.camera_rays(eyes, [0, 0, 0], TAN30, res, which=sample)
    o_ids, o_t = oracle_lib.first_hit(V, F, P, D, t_far, "bvh")
    check_rays(oracle_lib, V, F, P, D, g_ids, o_ids, o_t, t_far)
    g_vis = r.visible.cpu().numpy()
    g_ext = r.exterior.cpu().numpy()
    say(f"[gpu] visible {g_vis[:n_out].mean():.4f} of the shell, {g_vis[n_out:].sum()} inner")
    assert not g_vis[n_out:].any() and not g_ext[n_out:].any()
    assert g_vis[:n_out].mean() > 0.99 and g_ext[:n_out].all()
    assert np.array_equal(g_ext, oracle_lib.flood_fill(V, F, g_vis))
