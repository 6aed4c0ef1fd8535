"""Seeded synthetic meshes, atlases and normals for the normal bake.

The paper bakes from a raw marching-cubes mesh of roughly one million faces onto
a simplified, UV-unwrapped mesh (Sec. 6 "Geometry post-processing", Sec. 6.4
"Normal Map Baking").  Its assets, xatlas UVs and renderer are not available, so
displaced icospheres with a per-face grid atlas stand in for them:

* icosphere: golden-ratio icosahedron, edge-midpoint subdivision, projected to
  the unit sphere.  Level L has 10*4**L + 2 vertices and 20*4**L faces.
* radial displacement r(u) of the unit direction u: an analytic ripple, a seeded
  lattice gradient noise with quintic fade, and seeded Gaussian bumps.
* high-poly vertex normals: area-weighted sum of incident face normals.
* atlas: one right-triangle chart per face, packed in a square grid with a
  2-texel padding.

Everything is deterministic in its seed.  Positions are computed in float64 and
rounded to float32 once, at the end, because the bake consumes float32 inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from functools import lru_cache

import numpy as np

# ---------------------------------------------------------------------------
# Icosphere
# ---------------------------------------------------------------------------

_PHI = (1.0 + math.sqrt(5.0)) / 2.0

# Fixed vertex order of the base icosahedron (before projection to the sphere).
_ICO_V = np.array(
    [
        (-1, _PHI, 0), (1, _PHI, 0), (-1, -_PHI, 0), (1, -_PHI, 0),
        (0, -1, _PHI), (0, 1, _PHI), (0, -1, -_PHI), (0, 1, -_PHI),
        (_PHI, 0, -1), (_PHI, 0, 1), (-_PHI, 0, -1), (-_PHI, 0, 1),
    ],
    dtype=np.float64,
)
# Faces, counter-clockwise seen from outside (outward normals).
_ICO_F = np.array(
    [
        (0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
        (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
        (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
        (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1),
    ],
    dtype=np.int64,
)


def _subdivide(V: np.ndarray, F: np.ndarray):
    """One edge-midpoint subdivision step.

    New vertices are appended in creation order: faces in order, and within a
    face the edges (a,b), (b,c), (c,a).  A shared edge creates its midpoint the
    first time it is met.  Face (a,b,c) is replaced by
    [a,ab,ca], [ab,b,bc], [ca,bc,c], [ab,bc,ca] in that order.
    """
    nv = V.shape[0]
    n = F.shape[0]
    E = np.stack([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=1).reshape(-1, 2)
    lo = np.minimum(E[:, 0], E[:, 1])
    hi = np.maximum(E[:, 0], E[:, 1])
    key = lo * nv + hi
    _, first, inv = np.unique(key, return_index=True, return_inverse=True)
    order = np.argsort(first, kind="stable")  # unique edges in creation order
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    mids = nv + rank[inv.reshape(-1)]
    ab, bc, ca = mids.reshape(n, 3).T
    ue = order  # index into the unique set, creation-ordered
    first_e = E[first[ue]]
    M = V[first_e[:, 0]] + V[first_e[:, 1]]
    M /= np.linalg.norm(M, axis=1, keepdims=True)
    a, b, c = F[:, 0], F[:, 1], F[:, 2]
    Fn = np.stack(
        [
            np.stack([a, ab, ca], 1),
            np.stack([ab, b, bc], 1),
            np.stack([ca, bc, c], 1),
            np.stack([ab, bc, ca], 1),
        ],
        axis=1,
    ).reshape(-1, 3)
    return np.concatenate([V, M], axis=0), Fn


@lru_cache(maxsize=8)
def _icosphere_cached(level: int):
    V = _ICO_V / np.linalg.norm(_ICO_V, axis=1, keepdims=True)
    F = _ICO_F.copy()
    for _ in range(level):
        V, F = _subdivide(V, F)
    V.setflags(write=False)
    F.setflags(write=False)
    return V, F


def icosphere(level: int):
    """Unit icosphere of the given level: (V float64 [10*4^L+2, 3], F int64 [20*4^L, 3])."""
    if level < 0 or level > 10:
        raise ValueError("icosphere level must be in [0, 10]")
    V, F = _icosphere_cached(level)
    return V, F


# ---------------------------------------------------------------------------
# Radial displacements of the unit direction u
# ---------------------------------------------------------------------------

def unit_directions(V: np.ndarray) -> np.ndarray:
    V = np.asarray(V, dtype=np.float64)
    return V / np.linalg.norm(V, axis=1, keepdims=True)


def _theta_phi(U: np.ndarray):
    theta = np.arccos(np.clip(U[:, 2], -1.0, 1.0))
    phi = np.arctan2(U[:, 1], U[:, 0])
    return theta, phi


def analytic_radius(U: np.ndarray, amp: float = 0.02) -> np.ndarray:
    """r = 1 + amp*sin(6 theta)*cos(5 phi), theta = arccos(z), phi = atan2(y, x)."""
    th, ph = _theta_phi(U)
    return 1.0 + amp * np.sin(6.0 * th) * np.cos(5.0 * ph)


def analytic_normal(U: np.ndarray, amp: float = 0.02) -> np.ndarray:
    """Closed-form unit normal of the surface r(theta, phi)*u for the ripple above.

    With S = r u, dS/dtheta x dS/dphi = r sin(theta) (r u - r_theta e_theta -
    (r_phi / sin theta) e_phi).  Undefined at the poles (sin theta = 0), where
    the ripple has a kink.
    """
    th, ph = _theta_phi(U)
    st, ct = np.sin(th), np.cos(th)
    sp, cp = np.sin(ph), np.cos(ph)
    r = 1.0 + amp * np.sin(6 * th) * np.cos(5 * ph)
    r_t = 6.0 * amp * np.cos(6 * th) * np.cos(5 * ph)
    r_p = -5.0 * amp * np.sin(6 * th) * np.sin(5 * ph)
    u = np.stack([st * cp, st * sp, ct], 1)
    e_t = np.stack([ct * cp, ct * sp, -st], 1)
    e_p = np.stack([-sp, cp, np.zeros_like(sp)], 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        n = r[:, None] * u - r_t[:, None] * e_t - (r_p / st)[:, None] * e_p
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def _fade(t):
    # quintic fade 6t^5 - 15t^4 + 10t^3 (C2 continuous)
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


class _NoiseTable:
    """Seeded permutation + gradient table for 3D lattice gradient noise."""

    def __init__(self, seed: int):
        rng = np.random.default_rng([int(seed), 0x6E6F6973])
        perm = rng.permutation(256).astype(np.int64)
        self.perm = np.concatenate([perm, perm])
        g = rng.normal(size=(256, 3))
        self.grad = g / np.linalg.norm(g, axis=1, keepdims=True)

    def hash3(self, ix, iy, iz):
        p = self.perm
        return p[p[p[ix & 255] + (iy & 255)] + (iz & 255)]


def gradient_noise(P: np.ndarray, seed: int) -> np.ndarray:
    """One octave of seeded 3D lattice gradient noise at points P [n, 3].

    At each of the 8 surrounding lattice corners a hashed unit gradient is dotted
    with the offset to the point; the 8 values are blended trilinearly with the
    quintic fade.  Zero at lattice points.
    """
    tab = _NoiseTable(seed)
    P = np.asarray(P, dtype=np.float64)
    base = np.floor(P)
    f = P - base
    bi = base.astype(np.int64)
    w = _fade(f)
    out = np.zeros(P.shape[0])
    for dx in (0, 1):
        wx = w[:, 0] if dx else 1.0 - w[:, 0]
        for dy in (0, 1):
            wy = w[:, 1] if dy else 1.0 - w[:, 1]
            for dz in (0, 1):
                wz = w[:, 2] if dz else 1.0 - w[:, 2]
                h = tab.hash3(bi[:, 0] + dx, bi[:, 1] + dy, bi[:, 2] + dz)
                g = tab.grad[h]
                off = f - np.array([dx, dy, dz], dtype=np.float64)
                out += wx * wy * wz * np.einsum("ij,ij->i", g, off)
    return out


def noise_radius(U: np.ndarray, seed: int, octaves: int, amp: float,
                 base_freq: float = 3.0, persistence: float = 0.5) -> np.ndarray:
    """r = 1 + sum_k amp*persistence^k * noise(base_freq*2^k * u)."""
    r = np.ones(U.shape[0])
    for k in range(octaves):
        r += amp * persistence ** k * gradient_noise(U * (base_freq * 2.0 ** k), seed)
    return r


def bump_centres(n_bumps: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng([int(seed), 0x62756D70])
    c = rng.normal(size=(n_bumps, 3))
    return c / np.linalg.norm(c, axis=1, keepdims=True)


def bump_radius(U: np.ndarray, seed: int, n_bumps: int = 32, height: float = 0.05,
                sigma: float = 0.05) -> np.ndarray:
    """Sum of Gaussian bumps height*exp(-|u - c|^2 / (2 sigma^2)) (chord distance)."""
    C = bump_centres(n_bumps, seed)
    out = np.zeros(U.shape[0])
    for c in C:
        d2 = np.sum((U - c) ** 2, axis=1)
        out += height * np.exp(-d2 / (2.0 * sigma * sigma))
    return out


def displace(V_unit: np.ndarray, radius: np.ndarray) -> np.ndarray:
    return (V_unit * radius[:, None]).astype(np.float32)


# ---------------------------------------------------------------------------
# Normals, atlas, decimation
# ---------------------------------------------------------------------------

def vertex_normals(V: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Area-weighted unit vertex normals (sum of unnormalised face cross products).

    Used to give the high-poly input its smooth normals.  Float64 accumulation,
    float32 result.  Vertices with a zero sum get (0, 0, 0).
    """
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    c = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    nv = V.shape[0]
    idx = F.reshape(-1)
    acc = np.empty((nv, 3))
    for k in range(3):
        w = np.repeat(c[:, k], 3)
        acc[:, k] = np.bincount(idx, weights=w, minlength=nv)
    ln = np.linalg.norm(acc, axis=1, keepdims=True)
    with np.errstate(invalid="ignore", divide="ignore"):
        n = np.where(ln > 0, acc / np.where(ln > 0, ln, 1.0), 0.0)
    return n.astype(np.float32)


def grid_side(n_faces: int) -> int:
    """G = ceil(sqrt(n_faces)), exact in integers."""
    if n_faces <= 0:
        return 0
    return math.isqrt(n_faces - 1) + 1


def face_grid_atlas(n_faces: int, res: int, pad_texels: float = 2.0) -> np.ndarray:
    """Per-corner UVs [n_faces, 3, 2] float32: one right-triangle chart per face.

    G = ceil(sqrt(F)) cells per side, cell side s = res / G texels (a real
    number), padding p = min(pad, s / 4).  Face f sits in cell (f mod G, f div G)
    with corners (x0+p, y0+p), (x0+s-p, y0+p), (x0+p, y0+s-p) in texel units,
    u = x / res, v = y / res.
    """
    G = grid_side(n_faces)
    s = res / G
    p = min(pad_texels, s / 4.0)
    f = np.arange(n_faces)
    x0 = (f % G) * s
    y0 = (f // G) * s
    uv = np.empty((n_faces, 3, 2), dtype=np.float64)
    uv[:, 0, 0] = x0 + p
    uv[:, 0, 1] = y0 + p
    uv[:, 1, 0] = x0 + s - p
    uv[:, 1, 1] = y0 + p
    uv[:, 2, 0] = x0 + p
    uv[:, 2, 1] = y0 + s - p
    return (uv / res).astype(np.float32)


def sphere_viewpoints(n: int, center, radius: float) -> np.ndarray:
    """n points spread over the sphere of the given centre and radius
    (Fibonacci spiral: z_k = 1 - (2k + 1)/n, longitude k times the golden
    angle), float32 [n, 3]: camera positions around a mesh."""
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    P = np.stack([rho * np.cos(phi), rho * np.sin(phi), z], 1) * radius + np.asarray(center, np.float64)
    return P.astype(np.float32)


def hidden_face_mesh(outer_level: int = 5, inner_level: int = 3, inner_scale: float = 0.55, seed: int = 7):
    """A closed noise-displaced shell (icosphere outer_level) enclosing a
    smaller sphere (icosphere inner_level) that no exterior viewpoint sees:
    20,480 + 1,280 = 21,760 faces at the defaults, the size of the generated
    meshes the hidden-face pass runs on.  Returns float32 V, int32 F and the
    number of shell faces (the shell's faces come first)."""
    Vo, Fo = icosphere(outer_level)
    U = unit_directions(Vo)
    Vo = displace(U, noise_radius(U, seed, 4, 0.03))
    Vi, Fi = icosphere(inner_level)
    Vi = (Vi * inner_scale).astype(np.float32)
    V = np.concatenate([Vo.astype(np.float32), Vi])
    F = np.concatenate([Fo, Fi + Vo.shape[0]]).astype(np.int32)
    return V, F, Fo.shape[0]


def texture_views(radius: float) -> np.ndarray:
    """The ten generated views of the paper's texturing (front, rear, top,
    bottom, +-45 deg frontal, left, right, +-45 deg rear) as camera positions
    on a circle / the poles of the given radius, y up, front = +z; float32 [10, 3]."""
    s = radius * math.sqrt(0.5)
    P = [(0, 0, radius), (0, 0, -radius), (0, radius, 0), (0, -radius, 0), (s, 0, s), (-s, 0, s),
         (radius, 0, 0), (-radius, 0, 0), (s, 0, -s), (-s, 0, -s)]
    return np.array(P, np.float32)


def textured_bumpy_mesh(level: int = 5, res: int = 2048, seed: int = 3):
    """An icosphere displaced by 4-octave noise and 32 Gaussian bumps (which
    occlude each other at grazing views), with the per-face grid atlas:
    float32 V, int32 F, float32 per-corner UV [F, 3, 2]."""
    V, F = icosphere(level)
    U = unit_directions(V)
    Vd = displace(U, noise_radius(U, seed, 4, 0.03) + bump_radius(U, seed + 1, 32, 0.08, 0.06))
    return Vd.astype(np.float32), F.astype(np.int32), face_grid_atlas(F.shape[0], res)


def decimate(V: np.ndarray, F: np.ndarray, n_target: int, seed: int):
    """Delete uniformly random faces (seeded) down to n_target, then drop
    unreferenced vertices keeping the order of the rest."""
    F = np.asarray(F)
    if n_target >= F.shape[0]:
        return V, F
    rng = np.random.default_rng([int(seed), 0x64656369])
    keep = np.sort(rng.choice(F.shape[0], size=n_target, replace=False))
    Fk = F[keep]
    used = np.zeros(V.shape[0], dtype=bool)
    used[Fk.reshape(-1)] = True
    remap = np.cumsum(used) - 1
    return V[used], remap[Fk]


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

@dataclass
class Asset:
    """One bake problem: float32 / int32 arrays laid out as the bake consumes them."""
    name: str
    hi_V: np.ndarray   # [Vh, 3] f32
    hi_F: np.ndarray   # [Fh, 3] i32
    hi_N: np.ndarray   # [Vh, 3] f32
    lo_V: np.ndarray   # [Vl, 3] f32
    lo_F: np.ndarray   # [Fl, 3] i32
    lo_UV: np.ndarray  # [Fl, 3, 2] f32
    res: int
    max_dist: float
    meta: dict = field(default_factory=dict)

    def arrays(self):
        return (self.hi_V, self.hi_F, self.hi_N, self.lo_V, self.lo_F, self.lo_UV)


def _lo_sphere(level: int, res: int):
    V, F = icosphere(level)
    lo_V = V.astype(np.float32)
    lo_F = F.astype(np.int32)
    return lo_V, lo_F, face_grid_atlas(F.shape[0], res)


def _hi_from_radius(level: int, radius_fn):
    V, F = icosphere(level)
    U = unit_directions(V)
    hi_V = displace(U, radius_fn(U))
    hi_F = F.astype(np.int32)
    return hi_V, hi_F, vertex_normals(hi_V, hi_F)


def make_config(cfg: int, seed: int = 0) -> Asset:
    """The synthetic workloads the bake is measured on.

    1: hi L4 (5,120 tris) with the analytic ripple, lo L1 (80 tris), 128^2, 0.1.
    2: hi L8 (1,310,720) with 4-octave noise (f0 3, A 0.03, persistence 0.5),
       lo L5 (20,480), 2048^2, 0.12.
    3: hi L9 (5,242,880) with 6-octave noise (A 0.04) + 32 bumps (0.05, sigma
       0.05), lo L6 (81,920), 4096^2, 0.15.
    """
    if cfg == 1:
        hi = _hi_from_radius(4, lambda U: analytic_radius(U, 0.02))
        lo = _lo_sphere(1, 128)
        return Asset("ripple_L4_to_L1_128", *hi, *lo, res=128, max_dist=0.1)
    if cfg == 2:
        hi = _hi_from_radius(8, lambda U: noise_radius(U, seed, 4, 0.03))
        lo = _lo_sphere(5, 2048)
        return Asset(f"noise4_L8_to_L5_2048_s{seed}", *hi, *lo, res=2048, max_dist=0.12)
    if cfg == 3:
        hi = _hi_from_radius(
            9, lambda U: noise_radius(U, seed, 6, 0.04) + bump_radius(U, seed) )
        lo = _lo_sphere(6, 4096)
        return Asset(f"noise6bumps_L9_to_L6_4096_s{seed}", *hi, *lo, res=4096, max_dist=0.15)
    raise ValueError(f"unknown config {cfg}")


CONFIGS = {
    1: dict(hi_level=4, lo_level=1, res=128, max_dist=0.1),
    2: dict(hi_level=8, lo_level=5, res=2048, max_dist=0.12),
    3: dict(hi_level=9, lo_level=6, res=4096, max_dist=0.15),
}


def _level_for(n_faces: int) -> int:
    """Smallest icosphere level with at least n_faces faces (20*4^L >= n)."""
    L = 0
    while 20 * 4 ** L < n_faces:
        L += 1
    return L


def batch_asset_specs(n_assets: int = 64, seed: int = 0, hi_range=(50_000, 2_000_000),
                      lo_range=(1_300, 40_000), res_choices=(512, 1024, 2048),
                      max_dist: float = 0.1) -> list:
    """Sizes of the uneven multi-asset batch: (index, hi faces, lo faces, res,
    max_dist) per asset, face counts log-uniform in the given ranges."""
    rng = np.random.default_rng([int(seed), 0x62617463])
    out = []
    for i in range(n_assets):
        nh = int(round(math.exp(rng.uniform(math.log(hi_range[0]), math.log(hi_range[1])))))
        nl = int(round(math.exp(rng.uniform(math.log(lo_range[0]), math.log(lo_range[1])))))
        res = int(rng.choice(res_choices))
        out.append((i, nh, nl, res, float(max_dist)))
    return out


def make_batch_asset(spec) -> Asset:
    """One asset of the batch: noise seed i (4 octaves, A 0.03) on the icosphere
    of the nearest level at or above the face count, randomly decimated down
    to it."""
    i, nh, nl, res, max_dist = spec
    Lh, Ll = _level_for(nh), _level_for(nl)
    V, F = icosphere(Lh)
    U = unit_directions(V)
    hV = displace(U, noise_radius(U, i, 4, 0.03))
    hV, hF = decimate(hV, F, nh, seed=1000 + i)
    hF = hF.astype(np.int32)
    lV, lF = icosphere(Ll)
    lV, lF = decimate(lV.astype(np.float32), lF, nl, seed=2000 + i)
    lF = lF.astype(np.int32)
    return Asset(f"batch{i}", hV, hF, vertex_normals(hV, hF), lV, lF,
                 face_grid_atlas(lF.shape[0], res), res=res, max_dist=max_dist,
                 meta=dict(hi_level=Lh, lo_level=Ll))


def make_batch_assets(n_assets: int = 64, seed: int = 0, hi_range=(50_000, 2_000_000),
                      lo_range=(1_300, 40_000), res_choices=(512, 1024, 2048),
                      max_dist: float = 0.1, workers: int = 1) -> list:
    """Uneven multi-asset batch (batch_asset_specs + make_batch_asset); with
    workers > 1 the assets are generated in a process pool."""
    specs = batch_asset_specs(n_assets, seed, hi_range, lo_range, res_choices, max_dist)
    if workers <= 1:
        return [make_batch_asset(sp) for sp in specs]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(make_batch_asset, specs, chunksize=1)
