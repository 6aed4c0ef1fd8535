"""Input generator checks: counts, topology, orientation, determinism."""
import numpy as np
import pytest

from synth import meshes as M


@pytest.mark.parametrize("level", range(0, 7))
def test_icosphere_counts_closed_manifold_outward(level):
    V, F = M.icosphere(level)
    assert V.shape == (10 * 4 ** level + 2, 3)
    assert F.shape == (20 * 4 ** level, 3)
    assert np.allclose(np.linalg.norm(V, axis=1), 1.0, atol=1e-12)
    # every directed edge exactly once and its reverse exactly once: closed,
    # manifold and consistently oriented
    E = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    key = E[:, 0] * V.shape[0] + E[:, 1]
    rkey = E[:, 1] * V.shape[0] + E[:, 0]
    assert np.unique(key).size == key.size
    assert np.array_equal(np.sort(key), np.sort(rkey))
    c = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    assert np.all(np.einsum("ij,ij->i", c, V[F].mean(1)) > 0)


def test_large_level_counts_match_config_shapes():
    # the differentiation workload's gradients are [10,242 x 3] and [655,362 x 3]
    assert M.icosphere(5)[0].shape[0] == 10242
    assert M.icosphere(8)[0].shape[0] == 655362
    assert M.icosphere(8)[1].shape[0] == 1310720


def test_noise_deterministic_and_seeded():
    U = M.unit_directions(M.icosphere(3)[0])
    a = M.gradient_noise(U * 3.0, 0)
    b = M.gradient_noise(U * 3.0, 0)
    c = M.gradient_noise(U * 3.0, 1)
    assert np.array_equal(a, b)
    assert not np.allclose(a, c)
    # gradient noise vanishes on the integer lattice
    P = np.array([[0.0, 0, 0], [1, 2, 3], [-2, 5, 7]])
    assert np.allclose(M.gradient_noise(P, 0), 0.0)
    assert np.abs(a).max() < 1.5


def test_analytic_normal_matches_finite_difference_surface():
    # closed-form normal of r(theta, phi) u against a finite-difference cross product
    th, ph = 0.9, 0.4
    amp = 0.02

    def S(t, p):
        u = np.array([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)])
        return (1 + amp * np.sin(6 * t) * np.cos(5 * p)) * u

    h = 1e-6
    St = (S(th + h, ph) - S(th - h, ph)) / (2 * h)
    Sp = (S(th, ph + h) - S(th, ph - h)) / (2 * h)
    n = np.cross(St, Sp)
    n /= np.linalg.norm(n)
    u = np.array([[np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)]])
    assert np.allclose(M.analytic_normal(u, amp)[0], n, atol=1e-8)


def test_atlas_layout():
    uv = M.face_grid_atlas(80, 128)
    assert uv.shape == (80, 3, 2) and uv.dtype == np.float32
    assert uv.min() >= 0 and uv.max() <= 1
    G = M.grid_side(80)
    assert G == 9
    s = 128 / G
    # right angle at corner 0, legs along +u and +v, padding 2 texels
    assert np.allclose(uv[:, 1, 1], uv[:, 0, 1]) and np.allclose(uv[:, 2, 0], uv[:, 0, 0])
    assert np.allclose((uv[:, 1, 0] - uv[:, 0, 0]) * 128, s - 4, atol=1e-4)
    # charts lie in disjoint cells
    cell = np.floor(uv.mean(1) * 128 / s).astype(int)
    assert np.unique(cell[:, 1] * G + cell[:, 0]).size == 80


def test_decimate():
    V, F = M.icosphere(3)
    V2, F2 = M.decimate(V, F, 700, seed=3)
    assert F2.shape == (700, 3)
    assert F2.max() == V2.shape[0] - 1
    assert np.unique(F2).size == V2.shape[0]
    V3, F3 = M.decimate(V, F, 700, seed=3)
    assert np.array_equal(F2, F3)


def test_config_shapes_small():
    a = M.make_config(1)
    assert a.hi_V.shape == (2562, 3) and a.hi_F.shape == (5120, 3)
    assert a.lo_V.shape == (42, 3) and a.lo_F.shape == (80, 3)
    assert a.lo_UV.shape == (80, 3, 2) and a.res == 128 and a.max_dist == 0.1
    assert a.hi_V.dtype == np.float32 and a.hi_F.dtype == np.int32
    assert np.allclose(np.linalg.norm(a.hi_N, axis=1), 1, atol=1e-6)


# ---- the simplification's shapes ------------------------------------------

def _edge_counts(F):
    import numpy as np
    F = np.asarray(F, np.int64)
    e = np.sort(np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]]), axis=1)
    _, c = np.unique(e, axis=0, return_counts=True)
    return c


def test_closed_shapes_are_oriented_genus_zero_manifolds():
    import numpy as np
    from synth import shapes as S
    for V, F in (S.cube_grid(1), S.cube_grid(4), S.tetrahedron(), S.bipyramid(), S.octahedron(),
                 S.noisy_sphere(2, seed=1)):
        V = np.asarray(V, np.float64)
        c = _edge_counts(F)
        assert (c == 2).all()
        assert V.shape[0] - c.size + F.shape[0] == 2
        a, b, d = (V[np.asarray(F)[:, k]] for k in range(3))
        n = np.cross(b - a, d - a)
        centre = V.mean(0)
        assert ((n * ((a + b + d) / 3 - centre)).sum(1) > 0).all()    # outward (star-shaped shapes)


def test_cube_grid_and_patch_counts():
    import numpy as np
    from synth import shapes as S
    V, F = S.cube_grid(3)
    assert V.shape == (6 * 9 + 2, 3) and F.shape == (12 * 9, 3)
    assert set(np.unique(V)) <= {0.0, 1 / 3, 2 / 3, 1.0}
    V, F = S.grid_patch(5, amp=0.2, seed=3)
    assert V.shape == (36, 3) and F.shape == (50, 3)
    c = _edge_counts(F)
    assert (c == 1).sum() == 4 * 5 and ((c == 1) | (c == 2)).all()   # the square's border


def test_simplify_inputs_are_seeded_and_sized():
    import numpy as np
    from synth import shapes as S
    V, F, target, name = S.simplify_input(0)
    V2, F2, _, _ = S.simplify_input(0)
    assert F.shape == (20480, 3) and target == 1000 and V.dtype == np.float32 and F.dtype == np.int32
    assert np.array_equal(V, V2) and np.array_equal(F, F2)
    assert not np.array_equal(V, S.simplify_input(0, seed=1)[0])
