"""Seeded synthetic meshes for the simplification pass.

Only inputs: closed and open triangle meshes with known geometry (a
triangulated cube, small polyhedra, height-field patches, noise-displaced
spheres).  No quadric, placement or collapse arithmetic lives here; the FP64
oracle and the GPU path both consume what it returns.
"""
from __future__ import annotations

import numpy as np

from .meshes import displace, icosphere, noise_radius, unit_directions


def cube_grid(n: int):
    """Axis-aligned unit cube [0,1]^3, each side an n x n grid of quads split
    into two triangles, outward facing: (V float64 [6n^2+2, 3], F int64 [12n^2, 3])."""
    if n < 1:
        raise ValueError("n >= 1")
    index = {}
    V = []

    def vid(p):
        key = tuple(int(round(c * n)) for c in p)
        if key not in index:
            index[key] = len(V)
            V.append([k / n for k in key])
        return index[key]

    F = []
    # each side: origin corner o, in-plane axes a, b with a x b pointing outward
    sides = []
    for axis in range(3):
        a, b = (axis + 1) % 3, (axis + 2) % 3
        for hi in (0, 1):
            o = np.zeros(3)
            o[axis] = hi
            ea, eb = np.zeros(3), np.zeros(3)
            ea[a], eb[b] = 1.0, 1.0
            if hi == 0:
                ea, eb = eb, ea
            sides.append((o, ea, eb))
    for o, ea, eb in sides:
        for i in range(n):
            for j in range(n):
                p00 = o + ea * (i / n) + eb * (j / n)
                p10 = o + ea * ((i + 1) / n) + eb * (j / n)
                p01 = o + ea * (i / n) + eb * ((j + 1) / n)
                p11 = o + ea * ((i + 1) / n) + eb * ((j + 1) / n)
                v00, v10, v01, v11 = vid(p00), vid(p10), vid(p01), vid(p11)
                F.append([v00, v10, v11])
                F.append([v00, v11, v01])
    return np.asarray(V, np.float64), np.asarray(F, np.int64)


def tetrahedron():
    V = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], np.float64)
    F = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]], np.int64)
    return V, F


def bipyramid():
    """Triangle a, b, c (0, 1, 2) in z = 0 with apexes n (3, z = 1) and s (4, z = -1)."""
    V = np.array([[1, 0, 0], [-0.5, 0.8660254037844386, 0], [-0.5, -0.8660254037844386, 0],
                  [0, 0, 1], [0, 0, -1]], np.float64)
    F = np.array([[3, 0, 1], [3, 1, 2], [3, 2, 0], [4, 1, 0], [4, 2, 1], [4, 0, 2]], np.int64)
    return V, F


def octahedron():
    V = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.float64)
    F = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4], [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]], np.int64)
    return V, F


def grid_patch(n: int, amp: float = 0.0, seed: int = 0):
    """Open square patch [0,1]^2 of n x n quads (two triangles each), heights
    z = amp * (seeded sum of three smooth bumps): (V [(n+1)^2, 3], F [2n^2, 3])."""
    rng = np.random.default_rng(seed)
    xs = np.linspace(0.0, 1.0, n + 1)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    Z = np.zeros_like(X)
    for _ in range(3):
        cx, cy, s = rng.random(), rng.random(), 0.15 + 0.2 * rng.random()
        Z += np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * s * s))
    V = np.stack([X.ravel(), Y.ravel(), (amp * Z).ravel()], 1)
    F = []
    for i in range(n):
        for j in range(n):
            a, b, c, d = i * (n + 1) + j, (i + 1) * (n + 1) + j, i * (n + 1) + j + 1, (i + 1) * (n + 1) + j + 1
            F.append([a, b, d])
            F.append([a, d, c])
    return V, np.asarray(F, np.int64)


def noisy_sphere(level: int, amp: float = 0.03, octaves: int = 4, seed: int = 0):
    """Icosphere of the given level displaced radially by seeded gradient noise
    (the shape family of the bake's high-poly inputs): float32 V, int32 F."""
    V0, F = icosphere(level)
    U = unit_directions(V0)
    V = displace(U, noise_radius(U, seed, octaves, amp))
    return V.astype(np.float32), F.astype(np.int32)


# Simplification workloads: (name, icosphere level, noise octaves, target faces)
SIMPLIFY_WORKLOADS = {
    0: ("noise4 icosphere L5 (20,480 tris) -> 1,000 tris", 5, 4, 1000),
    1: ("noise4 icosphere L6 (81,920 tris) -> 5,000 tris", 6, 4, 5000),
    2: ("noise4 icosphere L8 (1,310,720 tris) -> 10,000 tris", 8, 4, 10000),
    3: ("noise4 icosphere L8 (1,310,720 tris) -> 5,000 tris", 8, 4, 5000),
}


def simplify_input(cfg: int, seed: int = 0):
    """(V float32, F int32, target faces, description) of a simplification workload."""
    name, level, octaves, target = SIMPLIFY_WORKLOADS[cfg]
    V, F = noisy_sphere(level, 0.03, octaves, seed)
    return V, F, target, name
