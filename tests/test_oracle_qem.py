"""Pins of the FP64 simplification oracle (Sec. 6.1, quadric edge collapse with
edge-constrained optimal placement) against facts that do not come from the
oracle itself: squared distances to face planes, least squares, closed forms
of flat and axis-aligned geometry, the topology of small polyhedra, Euler's
formula, a brute-force rescan of the greedy order, and the round rule written
out over the oracle's per-edge values."""
import numpy as np
import pytest

import oracle
from synth import shapes as S

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def edges_of(F):
    E = {}
    for f in np.asarray(F):
        for a, b in ((f[0], f[1]), (f[1], f[2]), (f[2], f[0])):
            k = (min(a, b), max(a, b))
            E[k] = E.get(k, 0) + 1
    return E


def faces_around(F, v):
    return [i for i, f in enumerate(np.asarray(F)) if v in f]


def unit_planes(V, F, faces):
    """(n, d) with |n| = 1 and n.x + d = 0 on each face's plane."""
    out = []
    for i in faces:
        a, b, c = (np.asarray(V, np.float64)[k] for k in F[i])
        n = np.cross(b - a, c - a)
        n = n / np.linalg.norm(n)
        out.append((n, -n @ a))
    return out


def qform(q, x):
    """[x;1]^T Q [x;1] from the 4x4 matrix (not the oracle's expansion)."""
    M = np.array([[q[0], q[1], q[2], q[3]], [q[1], q[4], q[5], q[6]],
                  [q[2], q[5], q[7], q[8]], [q[3], q[6], q[8], q[9]]])
    h = np.append(x, 1.0)
    return h @ M @ h


# ------------------------------------------------------------------ quadrics

def test_quadric_is_the_sum_of_squared_plane_distances():
    V, F = S.noisy_sphere(2, amp=0.1, seed=3)
    Q = oracle.qem_quadrics(V, F)
    rng = np.random.default_rng(0)
    for v in rng.choice(V.shape[0], 20, replace=False):
        planes = unit_planes(V, F, faces_around(F, v))
        for x in rng.normal(size=(5, 3)):
            want = sum((n @ x + d) ** 2 for n, d in planes)
            assert qform(Q[v], x) == pytest.approx(want, rel=1e-10, abs=1e-12)


def test_quadric_of_a_cube_corner_counts_the_axis_planes():
    V, F = S.cube_grid(3)
    Q = oracle.qem_quadrics(V.astype(np.float32), F)
    v = int(np.nonzero((V == 0).all(1))[0][0])          # corner (0, 0, 0)
    around = [np.asarray(V)[F[i]] for i in faces_around(F, v)]
    k = [sum(1 for t in around if (t[:, ax] == 0).all()) for ax in range(3)]
    assert sum(k) == len(around) and min(k) >= 1
    for x in np.random.default_rng(1).normal(size=(6, 3)):
        assert qform(Q[v], x) == pytest.approx(k[0] * x[0] ** 2 + k[1] * x[1] ** 2 + k[2] * x[2] ** 2, rel=1e-12)


# ----------------------------------------------------------------- placement

def test_optimal_placement_is_the_least_squares_point_projected_onto_the_edge():
    V, F = S.noisy_sphere(2, amp=0.15, octaves=3, seed=5)
    E = oracle.qem_edges(V.astype(np.float64), F)
    V64 = V.astype(np.float64)
    checked = 0
    for (a, b), p, c in zip(E.edges, E.p, E.cost):
        planes = unit_planes(V, F, faces_around(F, a)) + unit_planes(V, F, faces_around(F, b))
        A = np.array([n for n, _ in planes]); rhs = -np.array([d for _, d in planes])
        G = A.T @ A
        w = np.linalg.eigvalsh(G)
        if w[0] * w[1] * w[2] < 1e-5 * w.sum() ** 3:      # keep clear of the singular branch
            continue
        x = np.linalg.lstsq(A, rhs, rcond=None)[0]
        d = V64[b] - V64[a]
        t = np.clip((x - V64[a]) @ d / (d @ d), 0.0, 1.0)
        want = (1 - t) * V64[a] + t * V64[b]
        np.testing.assert_allclose(p, want, atol=1e-9)
        assert c == pytest.approx(np.sum((A @ p - rhs) ** 2), rel=1e-8, abs=1e-14)
        checked += 1
    assert checked > 100


def test_flat_interior_edges_take_the_midpoint_at_zero_cost():
    V, F = S.grid_patch(6)                               # z = 0 everywhere: A is singular
    E = oracle.qem_edges(V, F)
    bnd = {v for e, k in edges_of(F).items() if k == 1 for v in e}
    inner = [i for i, (a, b) in enumerate(E.edges) if a not in bnd and b not in bnd]
    assert len(inner) > 20
    for i in inner:
        a, b = E.edges[i]
        np.testing.assert_array_equal(E.p[i], 0.5 * (V[a] + V[b]))
        assert E.cost[i] == 0.0


def test_boundary_rules():
    V, F = S.grid_patch(6, amp=0.3, seed=2)
    Q = oracle.qem_quadrics(V.astype(np.float32), F)
    V32 = V.astype(np.float32).astype(np.float64)
    E = oracle.qem_edges(V32, F)
    cnt = edges_of(F)
    bnd = {v for e, k in cnt.items() if k == 1 for v in e}
    seen = {"edge": 0, "one": 0, "both": 0}
    for i, (a, b) in enumerate(E.edges):
        q = Q[a] + Q[b]
        if cnt[(a, b)] == 1:                              # boundary edge: lower-error endpoint
            ea, eb = qform(q, V32[a]), qform(q, V32[b])
            want = V32[b] if eb < ea and not np.isclose(ea, eb, rtol=1e-9) else V32[a]
            if not np.isclose(ea, eb, rtol=1e-9):
                np.testing.assert_array_equal(E.p[i], want)
            seen["edge"] += 1
        elif (a in bnd) != (b in bnd):                    # boundary vertex stays put
            np.testing.assert_array_equal(E.p[i], V32[a] if a in bnd else V32[b])
            seen["one"] += 1
        elif a in bnd and b in bnd:                       # interior edge between boundaries
            assert not E.valid[i]
            seen["both"] += 1
    assert seen["edge"] > 10 and seen["one"] > 10


def test_midpoint_switch_places_interior_edges_at_the_midpoint():
    V, F = S.noisy_sphere(2, amp=0.1, seed=4)
    E = oracle.qem_edges(V.astype(np.float64), F, midpoint=True)
    V64 = V.astype(np.float64)
    np.testing.assert_array_equal(E.p, 0.5 * (V64[E.edges[:, 0]] + V64[E.edges[:, 1]]))


# ------------------------------------------------------------------ topology

def test_bipyramid_equator_edges_fail_the_link_condition():
    V, F = S.bipyramid()
    E = oracle.qem_edges(V, F)
    for (a, b), ok in zip(E.edges, E.valid):
        equator = a < 3 and b < 3
        assert ok == (not equator), (a, b)


def test_tetrahedron_edges_never_collapse():
    V, F = S.tetrahedron()
    E = oracle.qem_edges(V, F)
    assert len(E.edges) == 6 and not E.valid.any()


@pytest.mark.parametrize("method", ["greedy", "rounds"])
def test_octahedron_collapses_to_a_tetrahedron_and_stops(method):
    V, F = S.octahedron()
    r = oracle.qem_simplify(V.astype(np.float32), F, 4, method=method)
    assert r.F.shape[0] == 4 and r.V.shape[0] == 4
    assert all(k == 2 for k in edges_of(r.F).values())


@pytest.mark.parametrize("method", ["greedy", "rounds"])
@pytest.mark.parametrize("seed", [0, 3])
def test_simplified_sphere_stays_a_manifold_sphere_facing_out(method, seed):
    # mild noise (the bake inputs' amplitude): the fold rule is per face, so
    # rougher inputs can still end with a face folded over its neighbour at
    # this reduction; what must hold on any input is the topology
    V, F = S.noisy_sphere(4, amp=0.03, seed=seed)
    r = oracle.qem_simplify(V, F, 120, method=method)
    assert r.F.shape[0] == 120
    cnt = edges_of(r.F)
    assert all(k == 2 for k in cnt.values())                          # closed 2-manifold
    assert r.V.shape[0] - len(cnt) + r.F.shape[0] == 2                # Euler: genus 0
    assert len({tuple(sorted(f)) for f in r.F.tolist()}) == r.F.shape[0]
    a, b, c = (r.V[r.F[:, k]] for k in range(3))
    n = np.cross(b - a, c - a)
    assert ((n * (a + b + c)).sum(1) > 0).all()                       # no folded face (star-shaped input)


@pytest.mark.parametrize("method", ["greedy", "rounds"])
def test_triangulated_cube_simplifies_to_its_eight_corners(method):
    V, F = S.cube_grid(4)
    r = oracle.qem_simplify(V.astype(np.float32), F, 12, method=method)
    assert r.F.shape[0] == 12
    corners = {tuple(p) for p in np.round(r.V, 12).tolist()}
    assert corners == {(x, y, z) for x in (0.0, 1.0) for y in (0.0, 1.0) for z in (0.0, 1.0)}
    a, b, c = (r.V[r.F[:, k]] for k in range(3))
    n = np.cross(b - a, c - a)
    assert ((n * ((a + b + c) / 3 - 0.5)).sum(1) > 0).all()


# ------------------------------------------------------------------- drivers

def collapse_py(P, Q, F, a, b, p):
    """R6 written out: a survives at p with Q_a + Q_b; faces holding both go."""
    P = P.copy(); Q = Q.copy()
    P[a] = p
    Q[a] = Q[a] + Q[b]
    F = F.copy()
    F[F == b] = a
    keep = (F[:, 0] != F[:, 1]) & (F[:, 1] != F[:, 2]) & (F[:, 0] != F[:, 2])
    return P, Q, F[keep]


def compact(P, F):
    used = np.unique(F)
    remap = -np.ones(P.shape[0], np.int64)
    remap[used] = np.arange(used.size)
    return P[used], remap[F].astype(np.int32)


def test_greedy_heap_matches_a_brute_force_rescan():
    V, F = S.noisy_sphere(2, amp=0.12, seed=11)
    target = 60
    P = V.astype(np.float64); Q = oracle.qem_quadrics(V, F); Fc = F.astype(np.int64)
    while Fc.shape[0] > target:
        E = oracle.qem_edges(P, Fc, Q=Q)
        ok = E.valid & (E.faces <= Fc.shape[0] - target)
        if not ok.any():
            break
        idx = np.nonzero(ok)[0]
        best = min(idx, key=lambda i: (E.cost[i], E.edges[i][0], E.edges[i][1]))
        a, b = E.edges[best]
        P, Q, Fc = collapse_py(P, Q, Fc, a, b, E.p[best])
    want_V, want_F = compact(P, Fc)
    r = oracle.qem_simplify(V, F, target, method="greedy")
    np.testing.assert_array_equal(r.F, want_F)
    np.testing.assert_array_equal(r.V, want_V)


def one_round_py(P, Q, F, target, rho):
    """The round rule over the oracle's per-edge values."""
    E = oracle.qem_edges(P, F, Q=Q)
    bits = E.cost.astype(np.float32).view(np.uint32).astype(np.uint64)
    key = (bits << np.uint64(32)) | np.arange(len(E.edges), dtype=np.uint64)
    valid = np.nonzero(E.valid)[0]
    k = min(max(int(np.ceil(rho * valid.size)), 1), valid.size)
    tau = np.sort(bits[valid])[k - 1]
    elig = E.valid & (bits <= tau)
    big = np.uint64(2 ** 64 - 1)
    m = np.full(P.shape[0], big)
    for i in np.nonzero(elig)[0]:
        for v in E.edges[i]:
            m[v] = min(m[v], key[i])
    M = m.copy()
    for a, b in E.edges:
        M[a] = min(M[a], m[b]); M[b] = min(M[b], m[a])
    win = [i for i in np.nonzero(elig)[0] if M[E.edges[i][0]] == key[i] and M[E.edges[i][1]] == key[i]]
    budget = F.shape[0] - target
    if sum(E.faces[i] for i in win) > budget:
        win.sort(key=lambda i: key[i])
        keep, cum = [], 0
        for i in win:
            if cum + E.faces[i] > budget:
                break
            keep.append(i); cum += E.faces[i]
        win = keep
    for i in win:
        a, b = E.edges[i]
        P, Q, F = collapse_py(P, Q, F, a, b, E.p[i])
    return P, Q, F, len(win)


@pytest.mark.parametrize("target,rho,rounds", [(300, 0.25, 1), (300, 1.0, 1), (600, 0.5, 3), (1200, 1.0, 2)])
def test_rounds_match_the_round_rule_written_out(target, rho, rounds):
    V, F = S.noisy_sphere(3, amp=0.1, seed=2)                        # 1280 faces
    P = V.astype(np.float64); Q = oracle.qem_quadrics(V, F); Fc = F.astype(np.int64)
    for _ in range(rounds):
        if Fc.shape[0] <= target:
            break
        P, Q, Fc, n = one_round_py(P, Q, Fc, target, rho)
    want_V, want_F = compact(P, Fc)
    r = oracle.qem_simplify(V, F, target, method="rounds", rho=rho, max_rounds=rounds)
    np.testing.assert_array_equal(r.F, want_F)
    np.testing.assert_array_equal(r.V, want_V)
    if target == 1200:
        assert r.F.shape[0] == 1200          # the budget cut kept the cheapest prefix only


# ------------------------------------------------------------------- quality

def test_optimal_placement_beats_the_midpoint_and_rounds_track_greedy():
    V, F, target, _ = S.simplify_input(0)
    res = {}
    for name, kw in (("greedy", dict(method="greedy")), ("rounds", dict(method="rounds")),
                     ("midpoint", dict(method="rounds", midpoint=True))):
        r = oracle.qem_simplify(V, F, target, **kw)
        assert r.F.shape[0] == target
        res[name] = oracle.mesh_distance(V, F, r.V, r.F, n=3000)
    assert res["rounds"][0] < res["midpoint"][0]                      # Chamfer
    assert res["rounds"][1] < res["midpoint"][1]                      # Hausdorff
    assert res["rounds"][0] < 1.1 * res["greedy"][0]
    assert res["rounds"][1] < 1.25 * res["greedy"][1]


@pytest.mark.parametrize("method", ["greedy", "rounds"])
def test_rough_sphere_keeps_its_topology(method):
    V, F = S.noisy_sphere(4, amp=0.1, seed=7)
    r = oracle.qem_simplify(V, F, 120, method=method)
    cnt = edges_of(r.F)
    assert r.F.shape[0] == 120 and all(k == 2 for k in cnt.values())
    assert r.V.shape[0] - len(cnt) + r.F.shape[0] == 2
