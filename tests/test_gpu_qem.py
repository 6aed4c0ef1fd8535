"""GPU quadric edge-collapse simplification (Sec. 6.1) against the FP64
oracle, through the C ABI.  Both sides evaluate the same FP64 definitions, so
the per-edge values, the quadrics and every round's result must agree exactly:
the same edges, validity, face counts and placements; after any number of
rounds the same faces in the same order and the same vertices (the GPU's
float32 output equals the oracle's FP64 positions rounded to float32).  At the
full workload size (1.31M faces) the first round is compared with the oracle
run here, the whole runs to 10k and 5k faces with the oracle's stored result
(hashes of faces and vertices, per-round stats), and the run's invariants and
sampled distance to the input are checked too."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from synth import shapes as S  # noqa: E402


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


def dev(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x, dt)).to("cuda")


def edges_of(F):
    F = np.asarray(F, np.int64)
    e = np.sort(np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]]), axis=1)
    k, c = np.unique(e, axis=0, return_counts=True)
    return k, c


def gpu_simplify(B, V, F, target, **kw):
    say(f"[gpu] qem_simplify n_f={F.shape[0]} target={target} {kw}")
    r = B.qem_simplify(dev(V, np.float32), dev(F, np.int32), target, **kw)
    torch.cuda.synchronize()
    return r.V.cpu().numpy(), r.F.cpu().numpy(), r.rounds, r.stats


MESHES = {
    "sphere_L4": lambda: S.noisy_sphere(4, amp=0.05, seed=1),
    "rough_L3": lambda: S.noisy_sphere(3, amp=0.15, seed=2),
    "patch": lambda: tuple(np.asarray(x, t) for x, t in zip(S.grid_patch(12, amp=0.3, seed=4),
                                                             (np.float32, np.int32))),
    "cube": lambda: (S.cube_grid(5)[0].astype(np.float32), S.cube_grid(5)[1].astype(np.int32)),
    "flat": lambda: tuple(np.asarray(x, t) for x, t in zip(S.grid_patch(8), (np.float32, np.int32))),
}


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("midpoint", [False, True])
def test_edges_and_quadrics_match_the_oracle(B, oracle_lib, name, midpoint):
    V, F = MESHES[name]()
    say(f"[gpu] qem_edges {name} n_f={F.shape[0]} midpoint={midpoint}")
    g = B.qem_edges(dev(V, np.float32), dev(F, np.int32), midpoint=midpoint)
    torch.cuda.synchronize()
    o = oracle_lib.qem_edges(V.astype(np.float64), F, midpoint=midpoint)
    np.testing.assert_array_equal(g.edges.cpu().numpy(), o.edges)
    np.testing.assert_array_equal(g.faces.cpu().numpy(), o.faces)
    np.testing.assert_array_equal(g.valid.cpu().numpy(), o.valid)
    np.testing.assert_array_equal(g.Q.cpu().numpy(), oracle_lib.qem_quadrics(V, F))
    np.testing.assert_array_equal(g.cost.cpu().numpy(), o.cost)
    np.testing.assert_array_equal(g.p.cpu().numpy(), o.p)
    assert o.valid.sum() > 0


@pytest.mark.parametrize("name,target,rho,rounds", [
    ("sphere_L4", 2000, 0.25, 1), ("sphere_L4", 2000, 1.0, 1), ("sphere_L4", 600, 0.25, 6),
    ("sphere_L4", 5000, 1.0, 3), ("rough_L3", 100, 0.5, 1000), ("patch", 40, 0.25, 1000),
    ("cube", 12, 0.25, 1000), ("flat", 8, 1.0, 1000),
])
@pytest.mark.parametrize("midpoint", [False, True])
def test_rounds_match_the_oracle_exactly(B, oracle_lib, name, target, rho, rounds, midpoint):
    V, F = MESHES[name]()
    gV, gF, gr, gst = gpu_simplify(B, V, F, target, rho=rho, max_rounds=rounds, midpoint=midpoint)
    o = oracle_lib.qem_simplify(V, F, target, method="rounds", rho=rho, max_rounds=rounds, midpoint=midpoint)
    assert gr == o.rounds
    np.testing.assert_array_equal(gst, o.stats)
    np.testing.assert_array_equal(gF, o.F)
    np.testing.assert_array_equal(gV, o.V.astype(np.float32))
    if rounds == 1000:
        assert gF.shape[0] <= max(target + 1, 4) or gst[-1, 2] == 0


def test_workload_simplifies_exactly_like_the_oracle(B, oracle_lib):
    V, F, target, name = S.simplify_input(0)
    gV, gF, gr, gst = gpu_simplify(B, V, F, target)
    o = oracle_lib.qem_simplify(V, F, target, method="rounds")
    say(f"[gpu] {name}: {gr} rounds, {gF.shape[0]} faces")
    assert gF.shape[0] == target
    np.testing.assert_array_equal(gst, o.stats)
    np.testing.assert_array_equal(gF, o.F)
    np.testing.assert_array_equal(gV, o.V.astype(np.float32))


def test_cube_collapses_to_its_corners(B):
    V, F = MESHES["cube"]()
    gV, gF, _, _ = gpu_simplify(B, V, F, 12)
    assert gF.shape[0] == 12
    assert {tuple(p) for p in gV.tolist()} == {(x, y, z) for x in (0.0, 1.0) for y in (0.0, 1.0) for z in (0.0, 1.0)}


def test_target_at_or_above_the_face_count_returns_the_mesh(B):
    V, F = S.noisy_sphere(2, seed=3)
    gV, gF, gr, _ = gpu_simplify(B, V, F, F.shape[0])
    assert gr == 0
    np.testing.assert_array_equal(gF, F)
    np.testing.assert_array_equal(gV, V)
    # unreferenced vertices are dropped and faces renumbered
    V2 = np.concatenate([np.zeros((3, 3), np.float32), V])
    gV, gF, _, _ = gpu_simplify(B, V2, F + 3, 10 ** 6)
    np.testing.assert_array_equal(gF, F)
    np.testing.assert_array_equal(gV, V)


def test_empty_mesh(B):
    gV, gF, gr, _ = gpu_simplify(B, np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), 4)
    assert gV.shape == (0, 3) and gF.shape == (0, 3) and gr == 0


@pytest.mark.parametrize("fill", [None, 0x7F])
def test_bad_faces_are_reported(B, fill):
    # a bad face is replaced by a degenerate stand-in that joins no vertex's
    # face list; the workspace filled with a byte pattern first makes sure no
    # pass reads anything the call did not write
    V, F = S.noisy_sphere(1, seed=0)
    for bad in (np.array([[0, 1, V.shape[0]]]), np.array([[0, 1, -1]]), np.array([[2, 2, 3]])):
        say(f"[gpu] qem bad face {bad.tolist()} workspace fill {fill}")
        Fb = np.concatenate([F, bad])
        ws = None
        if fill is not None:
            ws = torch.full((B.qem_workspace_size(V.shape[0], Fb.shape[0]),), fill, dtype=torch.uint8, device="cuda")
        with pytest.raises(B.BakeError) as e:
            B.qem_simplify(dev(V, np.float32), dev(Fb, np.int32), 10, workspace=ws)
        assert e.value.code == B.BAKE_E_INDEX
        with pytest.raises(B.BakeError) as e:
            B.qem_edges(dev(V, np.float32), dev(Fb, np.int32), workspace=ws)
        assert e.value.code == B.BAKE_E_INDEX


def test_results_are_deterministic(B):
    V, F = S.noisy_sphere(6, seed=5)
    a = gpu_simplify(B, V, F, 3000)
    b = gpu_simplify(B, V, F, 3000)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


# ---- the full workload: 1.31M faces -> 10,000 --------------------------------

@pytest.fixture(scope="module")
def big():
    V, F, target, name = S.simplify_input(2)
    return V, F, target


def test_full_size_first_round_matches_the_oracle(B, oracle_lib, big):
    V, F, target = big
    gV, gF, gr, gst = gpu_simplify(B, V, F, target, max_rounds=1)
    o = oracle_lib.qem_simplify(V, F, target, method="rounds", max_rounds=1)
    say(f"[gpu] full size, first collapse round: {gst.tolist()}")
    np.testing.assert_array_equal(gst, o.stats)
    np.testing.assert_array_equal(gF, o.F)
    np.testing.assert_array_equal(gV, o.V.astype(np.float32))


def test_full_size_run_invariants_and_distance(B, oracle_lib, big):
    V, F, target = big
    gV, gF, gr, gst = gpu_simplify(B, V, F, target)
    say(f"[gpu] full size: {gr} rounds -> {gF.shape[0]} faces, {gV.shape[0]} vertices")
    assert gF.shape[0] == target
    k, c = edges_of(gF)
    assert (c == 2).all()                                        # closed 2-manifold
    assert gV.shape[0] - k.shape[0] + gF.shape[0] == 2           # genus 0 kept
    assert np.unique(np.sort(gF, 1), axis=0).shape[0] == gF.shape[0]
    # sampled two-sided distance to the input surface (the oracle's closest point)
    ch, hd = oracle_lib.mesh_distance(V, F, gV, gF, n=3000, seed=7)
    say(f"[gpu] full size distance: chamfer {ch:.5f} hausdorff {hd:.5f}")
    assert ch < 1e-3 and hd < 6e-3


@pytest.mark.parametrize("target", [10000, 5000])
def test_full_size_run_matches_the_oracle_golden(B, big, target):
    """The whole 81- and 92-round runs against the oracle's result stored by
    tests/golden/make_qem_golden.py (hashes of the faces and of the vertices
    rounded to float32, and the per-round stats)."""
    V, F, _ = big
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "qem_noise4_L8.json")
    g = json.load(open(path))["targets"][str(target)]
    gV, gF, gr, gst = gpu_simplify(B, V, F, target)
    assert gr == g["rounds"]
    np.testing.assert_array_equal(gst, np.asarray(g["stats"], np.int64))
    assert gF.shape[0] == g["faces"] and gV.shape[0] == g["vertices"]
    assert hashlib.sha256(np.ascontiguousarray(gF, np.int32).tobytes()).hexdigest() == g["sha256_F_int32"]
    assert hashlib.sha256(np.ascontiguousarray(gV, np.float32).tobytes()).hexdigest() == g["sha256_V_float32"]
