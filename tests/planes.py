"""Small hand-made meshes for pins: planar grids with UV = (x, y)."""
import numpy as np

from synth import Asset


def grid(n, z=lambda x, y: 0.0 * x, x0=0.0, y0=0.0, size=1.0):
    """n x n cells over [x0, x0+size]^2, two CCW triangles per cell:
    (v00, v10, v11) then (v00, v11, v01); returns float32 V, int32 F."""
    xs = x0 + size * np.arange(n + 1) / n
    X, Y = np.meshgrid(xs, xs)  # Y rows
    V = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], 1)
    V[:, 2] = z(V[:, 0], V[:, 1])
    F = []
    for i in range(n):
        for j in range(n):
            v00 = i * (n + 1) + j
            v10 = v00 + 1
            v01 = v00 + (n + 1)
            v11 = v01 + 1
            F.append((v00, v10, v11))
            F.append((v00, v11, v01))
    return V.astype(np.float32), np.array(F, np.int32)


def plane_uv(V, F):
    """Per-corner UV = (x, y) of the vertex."""
    return np.ascontiguousarray(V[F][:, :, :2]).astype(np.float32)


def plane_asset(hi_V, hi_F, hi_N, res=64, lo_n=8, max_dist=0.25):
    lo_V, lo_F = grid(lo_n)
    return Asset("plane", hi_V, hi_F, hi_N.astype(np.float32), lo_V, lo_F, plane_uv(lo_V, lo_F),
                 res=res, max_dist=max_dist)


def grid_cell_triangle(x, y, n):
    """Index of the triangle of grid(n) containing (x, y) strictly inside
    (points must not lie on cell borders or on the cell diagonal)."""
    j = np.floor(x * n).astype(np.int64)
    i = np.floor(y * n).astype(np.int64)
    fx = x * n - j
    fy = y * n - i
    lower = fx > fy  # below the diagonal v00 -> v11: triangle (v00, v10, v11)
    return 2 * (i * n + j) + np.where(lower, 0, 1)


def textured_plane(n=8, occluder=False):
    """Grid over [0,1]^2 at z = 0 with UV = (x / 2, y) (the atlas' left half);
    optionally a square occluder at z = 0.5 over [0.3, 0.6] x [0.2, 0.7] with
    its UVs in the right half."""
    V, F = grid(n)
    UV = np.stack([V[F][:, :, 0] / 2, V[F][:, :, 1]], 2)
    if occluder:
        Vo, Fo = grid(2, z=lambda x, y: 0.0 * x + 0.5)
        Vo[:, 0] = 0.3 + 0.3 * Vo[:, 0]
        Vo[:, 1] = 0.2 + 0.5 * Vo[:, 1]
        uvo = np.stack([0.5 + 0.5 * (Vo[Fo][:, :, 0] - 0.3) / 0.3, (Vo[Fo][:, :, 1] - 0.2) / 0.5], 2)
        V = np.concatenate([V, Vo])
        F = np.concatenate([F, Fo + (n + 1) ** 2])
        UV = np.concatenate([UV, uvo])
    return V.astype(np.float32), F.astype(np.int32), np.ascontiguousarray(UV, np.float32)

