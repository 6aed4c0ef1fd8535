"""FP64 CPU oracle for the normal bake -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never links or calls it, and it imports nothing
from the GPU package: the two share no code.

The arithmetic lives in ``oracle.c`` (plain C, FP64, OpenMP over rays); this
module only marshals numpy arrays and chains the steps in the order of the
paper's bake (Sec. 6.4 "Normal Map Baking"):

1. low-poly smooth vertex normals and per-face tangent frames / reliability;
2. UV-space rasterisation of the low-poly (texel -> face, barycentrics);
3. per texel a world position p and the interpolated smooth normal d;
4. nearest line hit on the high-poly within +-max_dist (brute force over
   every triangle, or the independent FP64 BVH pinned against it), under one
   of two hit rules.  "plain" is the plain definition: a triangle is hit when
   the line meets it (all barycentric weights of the crossing >= 0) and the
   winner minimises (|t|, index).  "robust" is the convention the GPU library
   implements: a triangle is hit when the weights are all >= -EDGE_EPS and the
   winner minimises (floor(|t| / w), index) with w = max_dist * 2^-20, so a
   line through a shared edge or vertex, or two surfaces at the same distance,
   resolve to the lower triangle index instead of to rounding noise;
5. barycentric high-poly normal, projection into the tangent frame, neutral
   (0,0,1) for misses / unreliable / uncovered texels;
6. chart dilation.

The hidden-face removal of Sec. 6.2 is here too: camera rays from viewpoints
around the mesh, the first hit of each on the mesh (same triangle test, one
sided), the per-face visibility mask, and the flood fill over shared edges
gated by the face normals (``camera_rays``, ``first_hit``, ``visibility``,
``flood_fill``; ``oracle.c`` states the readings).

Mesh simplification (Sec. 6.1) lives in ``qem.c``: per-vertex quadrics, the
edge-constrained optimal placement, a serial greedy driver and the parallel
round schedule (``qem_quadrics``, ``qem_edges``, ``qem_simplify``), and a
sampled surface distance between two meshes (``mesh_distance``) for the
quality comparisons the section makes.

Parity unpinned: none of the paper's own quality numbers (its 50-asset
benchmark) can be reproduced here; every other function has a pin in
``tests/test_oracle.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sysconfig
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "qem.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ST_MISS, ST_UNREL, ST_UNCOV = -1, -2, -3


def build(force: bool = True) -> str:
    """Compile oracle.c and qem.c with gcc (FP64, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-Wall", "-o", tmp, *_SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = C.CDLL(_LIB_PATH)
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def set_threads(n: int = 0) -> int:
    lib = _load()
    lib.orc_set_threads.restype = C.c_int
    return lib.orc_set_threads(C.c_int(n))


def _call(name, *args):
    lib = _load()
    fn = getattr(lib, name)
    fn.restype = C.c_int
    rc = fn(*args)
    if rc != 0:
        raise ValueError(f"oracle {name} failed ({rc})")


def lo_normals(V, F):
    V = _c(V, np.float32); F = _c(F, np.int32)
    n = np.zeros((V.shape[0], 3)); ok = np.zeros(V.shape[0], np.uint8)
    _call("orc_lo_normals", _p(V), C.c_int64(V.shape[0]), _p(F), C.c_int64(F.shape[0]), _p(n), _p(ok))
    return n, ok.astype(bool)


def face_frames(V, F, UV, res, vn_valid=None):
    V = _c(V, np.float32); F = _c(F, np.int32); UV = _c(UV, np.float32)
    nf = F.shape[0]
    T = np.zeros((nf, 3)); B = np.zeros((nf, 3)); h = np.zeros(nf, np.int8); rel = np.zeros(nf, np.uint8)
    vv = None if vn_valid is None else _c(vn_valid, np.uint8)
    _call("orc_face_frames", _p(V), C.c_int64(V.shape[0]), _p(F), C.c_int64(nf), _p(UV),
          C.c_int32(res), _p(vv), _p(T), _p(B), _p(h), _p(rel))
    return T, B, h, rel.astype(bool)


def raster(UV, res):
    UV = _c(UV, np.float32)
    face = np.zeros(res * res, np.int32); bary = np.zeros((res * res, 3))
    _call("orc_raster", _p(UV), C.c_int64(UV.shape[0]), C.c_int32(res), _p(face), _p(bary))
    return face, bary


def rays(V, F, vn, face, bary):
    V = _c(V, np.float32); F = _c(F, np.int32); vn = _c(vn, np.float64)
    face = _c(face, np.int32); bary = _c(bary, np.float64)
    n = face.shape[0]
    P = np.zeros((n, 3)); D = np.zeros((n, 3)); ok = np.zeros(n, np.uint8)
    _call("orc_rays", _p(V), _p(F), _p(vn), C.c_int64(n), _p(face), _p(bary), _p(P), _p(D), _p(ok))
    return P, D, ok.astype(bool)


RULES = {"plain": 0, "robust": 1}


def _rule(rule):
    if rule not in RULES:
        raise ValueError(f"rule must be one of {sorted(RULES)}, not {rule!r}")
    return C.c_int(RULES[rule])


N_EXCLUDE = 4  # triangle ids a query can skip per ray


def _exclude(exclude, n):
    """Per-ray triangle ids to skip: None, [n] or [n, k <= N_EXCLUDE] (-1: none)."""
    if exclude is None:
        return None
    e = np.asarray(exclude, np.int64)
    if e.ndim == 1:
        e = e[:, None]
    if e.ndim != 2 or e.shape[0] != n or e.shape[1] > N_EXCLUDE:
        raise ValueError(f"exclude must be [n] or [n, <= {N_EXCLUDE}], got {e.shape}")
    out = np.full((n, N_EXCLUDE), -1, np.int32)
    out[:, :e.shape[1]] = e
    return out


def query(hi_V, hi_F, P, D, max_dist, active=None, method="brute", rule="robust", exclude=None):
    """Nearest-|t| two-sided line hit: (id [-1 miss], t, beta[3]).

    rule="plain": the plain definition (all weights >= 0, winner min (|t|,
    index)); rule="robust": the edge tolerance and distance quantum of the GPU
    library's convention (oracle.c states both).  exclude: triangle ids to skip
    per ray ([n] or [n, k <= N_EXCLUDE], -1 none), for the comparator's
    runner-up queries."""
    hi_V = _c(hi_V, np.float32); hi_F = _c(hi_F, np.int32)
    P = _c(P, np.float64); D = _c(D, np.float64)
    n = P.shape[0]
    ids = np.zeros(n, np.int32); t = np.zeros(n); beta = np.zeros((n, 3))
    act = None if active is None else _c(active, np.uint8)
    ex = _exclude(exclude, n)
    if method == "brute":
        _call("orc_query_brute", _p(hi_V), _p(hi_F), C.c_int64(hi_F.shape[0]), C.c_int64(n), _p(P),
              _p(D), _p(act), C.c_double(max_dist), _rule(rule), _p(ex), _p(ids), _p(t), _p(beta))
    elif method == "bvh":
        _call("orc_query_bvh", _p(hi_V), C.c_int64(hi_V.shape[0]), _p(hi_F), C.c_int64(hi_F.shape[0]),
              C.c_int64(n), _p(P), _p(D), _p(act), C.c_double(max_dist), _rule(rule), _p(ex), _p(ids),
              _p(t), _p(beta))
    else:
        raise ValueError(method)
    return ids, t, beta


def closest(hi_V, hi_F, P, max_dist, active=None, method="brute"):
    """Closest point of the high-poly within max_dist: (id [-1 miss], distance,
    barycentric weights [3] of the closest point)."""
    hi_V = _c(hi_V, np.float32); hi_F = _c(hi_F, np.int32)
    P = _c(P, np.float64)
    n = P.shape[0]
    ids = np.zeros(n, np.int32); dist = np.zeros(n); w = np.zeros((n, 3))
    act = None if active is None else _c(active, np.uint8)
    fn = {"brute": "orc_closest_brute", "bvh": "orc_closest_bvh"}[method]
    _call(fn, _p(hi_V), _p(hi_F), C.c_int64(hi_F.shape[0]), C.c_int64(n), _p(P), _p(act),
          C.c_double(max_dist), _p(ids), _p(dist), _p(w))
    return ids, dist, w


def closest_check(hi_V, hi_F, P, g):
    """Distance from each P[r] to triangle g[r]."""
    hi_V = _c(hi_V, np.float32); hi_F = _c(hi_F, np.int32)
    P = _c(P, np.float64); g = _c(g, np.int32)
    dist = np.zeros(g.shape[0])
    _call("orc_closest_check", _p(hi_V), _p(hi_F), C.c_int64(g.shape[0]), _p(P), _p(g), _p(dist))
    return dist


def closest_near(hi_V, hi_F, P, ids, dist, delta, eps_exact=1e-12):
    """Per point: does a triangle other than ids[r] lie within delta of the
    winning distance dist[r] without being an exact tie (|difference| >
    eps_exact)?  Such points are near ties of the closest-point query."""
    hi_V = _c(hi_V, np.float32); hi_F = _c(hi_F, np.int32)
    P = _c(P, np.float64); ids = _c(ids, np.int32); dist = _c(dist, np.float64)
    out = np.zeros(P.shape[0], np.uint8)
    _call("orc_closest_near", _p(hi_V), _p(hi_F), C.c_int64(hi_F.shape[0]), C.c_int64(P.shape[0]), _p(P),
          _p(ids), _p(dist), C.c_double(delta), C.c_double(eps_exact), _p(out))
    return out.astype(bool)


def frame_ok(lo_face, D, Tf):
    lo_face = _c(lo_face, np.int32); D = _c(D, np.float64); Tf = _c(Tf, np.float64)
    ok = np.zeros(lo_face.shape[0], np.uint8)
    _call("orc_frame_ok", C.c_int64(lo_face.shape[0]), _p(lo_face), _p(D), _p(Tf), _p(ok))
    return ok.astype(bool)


def encode(hi_F, hi_N, lo_face, D, Tf, hf, beta, status):
    hi_F = _c(hi_F, np.int32); hi_N = _c(hi_N, np.float32); lo_face = _c(lo_face, np.int32)
    D = _c(D, np.float64); Tf = _c(Tf, np.float64); hf = _c(hf, np.int8); beta = _c(beta, np.float64)
    st = _c(status, np.int32).copy()
    n = lo_face.shape[0]
    out = np.zeros((n, 3))
    _call("orc_encode", _p(hi_F), _p(hi_N), C.c_int64(n), _p(lo_face), _p(D), _p(Tf), _p(hf),
          _p(beta), _p(st), _p(out))
    return out, st


def dilate(map_flat, level, res, passes):
    m = _c(map_flat, np.float64).copy(); lv = _c(level, np.uint8).copy()
    _call("orc_dilate", _p(m), _p(lv), C.c_int32(res), C.c_int32(passes))
    return m, lv


def plane_check(hi_V, hi_F, P, D, g):
    """Per (ray, triangle): plane crossing t, distance of the crossing from the
    triangle, smallest barycentric weight of the crossing."""
    hi_V = _c(hi_V, np.float32); hi_F = _c(hi_F, np.int32)
    P = _c(P, np.float64); D = _c(D, np.float64); g = _c(g, np.int32)
    n = g.shape[0]
    t = np.zeros(n); dl = np.zeros(n); bm = np.zeros(n)
    _call("orc_plane_check", _p(hi_V), _p(hi_F), C.c_int64(n), _p(P), _p(D), _p(g), _p(t), _p(dl), _p(bm))
    return t, dl, bm


EDGE_EPS = 1.0 / 16384.0  # relative edge tolerance of the hit rule (barycentric units)
T_QUANT_BITS = 20         # distance quantum w = max_dist * 2^-20


def t_quantum(max_dist):
    return max_dist * 2.0 ** -T_QUANT_BITS


@dataclass
class Bake:
    """Result of an oracle bake; per-texel arrays are flat [res*res(,3)]."""
    res: int
    max_dist: float
    face: np.ndarray        # covering lo face or -1
    bary: np.ndarray        # [res*res, 3]
    texels: np.ndarray      # the texels that were baked (covered, possibly sampled)
    P: np.ndarray           # [n, 3] ray origins for `texels`
    D: np.ndarray           # [n, 3] ray directions
    hit: np.ndarray         # [n] query result before encoding (-1 miss), -2 if not traced
    t: np.ndarray           # [n]
    beta: np.ndarray        # [n, 3]
    status: np.ndarray      # [res*res] final status (-3 uncovered; sampled runs: -4 not baked)
    map_raw: np.ndarray     # [res*res, 3] before dilation
    map: np.ndarray         # [res*res, 3] after dilation
    level: np.ndarray       # [res*res] dilation level (0 covered, k filled in pass k, 255 empty)


def bake(asset, method="brute", texels=None, dilate_passes=2, kind="ray", max_dist=None,
         rule="robust") -> Bake:
    """Oracle bake of a whole asset (or of a subset of covered texels).
    kind="ray": two-sided line query along the interpolated normal, under the
    hit rule `rule` ("robust": the GPU library's convention; "plain": the plain
    nearest hit);
    kind="closest": closest point of the high-poly (the paper's form), for
    which Bake.t holds the distance.  max_dist defaults to the asset's."""
    hi_V, hi_F, hi_N, lo_V, lo_F, lo_UV = asset.arrays()
    res = int(asset.res)
    md = float(asset.max_dist if max_dist is None else max_dist)
    vn, vn_ok = lo_normals(lo_V, lo_F)
    Tf, _, hf, rel = face_frames(lo_V, lo_F, lo_UV, res, vn_ok)
    face, bary = raster(lo_UV, res)
    covered = np.nonzero(face >= 0)[0]
    full = texels is None
    tex = covered if full else np.asarray(texels, dtype=np.int64)
    if not full and np.any(face[tex] < 0):
        raise ValueError("sampled texels must be covered")
    lf = face[tex]
    P, D, mok = rays(lo_V, lo_F, vn, lf, bary[tex])
    fok = frame_ok(lf, D, Tf)
    active = rel[lf] & mok & fok
    if kind == "ray":
        ids, t, beta = query(hi_V, hi_F, P, D, md, active=active, method=method, rule=rule)
    elif kind == "closest":
        ids, t, beta = closest(hi_V, hi_F, P, md, active=active, method=method)
    else:
        raise ValueError(kind)
    st = np.where(active, ids, ST_UNREL).astype(np.int32)
    out, st = encode(hi_F, hi_N, lf, D, Tf, hf, beta, st)
    ntex = res * res
    status = np.full(ntex, ST_UNCOV if full else -4, np.int32)
    status[face < 0] = ST_UNCOV
    status[tex] = st
    map_raw = np.zeros((ntex, 3)); map_raw[:, 2] = 1.0
    map_raw[tex] = out
    hit = np.where(active, ids, ST_UNREL).astype(np.int32)
    if full:
        level = np.where(face >= 0, 0, 255).astype(np.uint8)
        m, level = dilate(map_raw, level, res, dilate_passes)
    else:
        m, level = map_raw.copy(), np.where(face >= 0, 0, 255).astype(np.uint8)
    return Bake(res, md, face, bary, tex, P, D, hit, t, beta, status, map_raw, m, level)


def rgb8(map_flat):
    """RGB8 encoding c = clamp(floor((x + 1) * 127.5 + 0.5), 0, 255)."""
    c = np.floor((np.asarray(map_flat, np.float64) + 1.0) * 127.5 + 0.5)
    return np.clip(c, 0, 255).astype(np.uint8)


def _frozen_args(asset, face, bary, g, hf):
    return (_c(asset.lo_V, np.float32), _c(asset.lo_F, np.int32), _c(asset.lo_UV, np.float32),
            _c(asset.hi_V, np.float32), _c(asset.hi_F, np.int32), _c(asset.hi_N, np.float32),
            _c(face, np.int32), _c(bary, np.float64), _c(g, np.int32), _c(hf, np.int8))


def frozen_forward(asset, face, bary, g, hf):
    """Per-ray output with the texel's lo face and barycentrics, the hit
    triangle g and the handedness held fixed: (out [n,3], (t, beta1, beta2) [n,3])."""
    loV, loF, UV, hiV, hiF, hiN, face, bary, g, hf = _frozen_args(asset, face, bary, g, hf)
    n = face.shape[0]
    out = np.zeros((n, 3)); tb = np.zeros((n, 3))
    _call("orc_frozen_forward", _p(loV), C.c_int64(loV.shape[0]), _p(loF), C.c_int64(loF.shape[0]),
          _p(UV), C.c_int32(asset.res), _p(hiV), _p(hiF), _p(hiN), C.c_int64(n), _p(face), _p(bary),
          _p(g), _p(hf), _p(out), _p(tb))
    return out, tb


def adjoint(asset, face, bary, g, hf, grad_out, magnitudes=False, bnoise=None):
    """FP64 reverse mode of frozen_forward: given d(loss)/d(out) per ray,
    returns (d loss / d lo_V [Vl,3], d loss / d hi_N [Vh,3]); with
    magnitudes=True also, per entry, the summed magnitudes of the terms added
    into it (the scale a floating-point evaluation of the sums is accurate to).
    With bnoise [n] (a bound per ray on the perturbation of the hit weights
    beta1, beta2) also, per entry of d loss / d hi_N, the first-order bound of
    how far its terms move under such a perturbation (oracle.c, orc_adjoint)."""
    loV, loF, UV, hiV, hiF, hiN, face, bary, g, hf = _frozen_args(asset, face, bary, g, hf)
    go = _c(grad_out, np.float64)
    glo = np.zeros((loV.shape[0], 3)); ghi = np.zeros((hiV.shape[0], 3))
    alo = np.zeros((loV.shape[0], 3)) if magnitudes else None
    ahi = np.zeros((hiV.shape[0], 3)) if magnitudes else None
    bn = None if bnoise is None else _c(np.broadcast_to(np.asarray(bnoise, np.float64), (face.shape[0],)), np.float64)
    shi = np.zeros((hiV.shape[0], 3)) if bn is not None else None
    _call("orc_adjoint", _p(loV), C.c_int64(loV.shape[0]), _p(loF), C.c_int64(loF.shape[0]), _p(UV),
          C.c_int32(asset.res), _p(hiV), C.c_int64(hiV.shape[0]), _p(hiF), _p(hiN),
          C.c_int64(face.shape[0]), _p(face), _p(bary), _p(g), _p(hf), _p(go), _p(glo), _p(ghi),
          _p(alo), _p(ahi), _p(bn), _p(shi))
    out = (glo, ghi, alo, ahi) if magnitudes else (glo, ghi)
    return out + (shi,) if bn is not None else out


def adjoint_at(asset, hit, grad_map, magnitudes=False, bnoise=None):
    """Adjoint of a whole bake's pre-dilation map at a given hit selection:
    hit [res*res] (a bake's status per texel, >= 0 for hits: e.g. the GPU's
    own), grad_map [res*res, 3].  The texel -> face assignment and barycentrics
    are the rasteriser's (exact integers), h_f the face frames'.  bnoise: None,
    or a function of (texels, t [n]) giving the weight perturbation bound per
    hit texel (t: the FP64 crossing distance at that selection), see adjoint."""
    hit = np.asarray(hit).reshape(-1)
    face, bary = raster(asset.lo_UV, asset.res)
    tex = np.nonzero((face >= 0) & (hit >= 0))[0]
    _, ok = lo_normals(asset.lo_V, asset.lo_F)
    _, _, hf, _ = face_frames(asset.lo_V, asset.lo_F, asset.lo_UV, asset.res, ok)
    gm = np.asarray(grad_map, np.float64).reshape(-1, 3)[tex]
    f = face[tex]
    bn = None
    if bnoise is not None:
        _, tb = frozen_forward(asset, f, bary[tex], hit[tex], hf[f])
        bn = bnoise(tex, tb[:, 0])
    return adjoint(asset, f, bary[tex], hit[tex], hf[f], gm, magnitudes, bn)


def bake_adjoint(asset, ob, grad_map):
    """Adjoint of a whole bake's pre-dilation map: the hit texels of the oracle
    bake `ob` carry grad_map [res*res,3]; misses, unreliable and uncovered
    texels are constant and carry none."""
    hit = ob.hit >= 0
    st = ob.status[ob.texels]
    hit &= st >= 0
    tex = ob.texels[hit]
    face = ob.face[tex]
    _, ok = lo_normals(asset.lo_V, asset.lo_F)
    _, _, hf, _ = face_frames(asset.lo_V, asset.lo_F, asset.lo_UV, asset.res, ok)
    gm = np.asarray(grad_map, np.float64).reshape(-1, 3)[tex]
    return adjoint(asset, face, ob.bary[tex], ob.hit[hit], hf[face], gm)


# ---------------------------------------------------------------------------
# Hidden-face removal (Sec. 6.2)
# ---------------------------------------------------------------------------

def camera_rays(eyes, target, tan_half, res, which=None):
    """Origins and unit directions [n, 3] of the pixels' rays, ray index (v res
    + i) res + j: every ray of every view, or the rays listed in `which`
    (readings in oracle.c)."""
    eyes = _c(eyes, np.float32).reshape(-1, 3)
    tg = _c(np.asarray(target, np.float32), np.float64).reshape(3)  # the target is a float input
    if which is None:
        n = eyes.shape[0] * res * res
        P = np.zeros((n, 3)); D = np.zeros((n, 3))
        _call("orc_camera_rays", _p(eyes), C.c_int32(eyes.shape[0]), _p(tg), C.c_double(tan_half),
              C.c_int32(res), _p(P), _p(D))
        return P, D
    which = _c(which, np.int64).reshape(-1)
    assert which.size == 0 or (which.min() >= 0 and which.max() < eyes.shape[0] * res * res)
    P = np.zeros((which.size, 3)); D = np.zeros((which.size, 3))
    _call("orc_camera_rays_at", _p(eyes), _p(tg), C.c_double(tan_half), C.c_int32(res),
          C.c_int64(which.size), _p(which), _p(P), _p(D))
    return P, D


def first_hit(V, F, P, D, t_far, method="brute", rule="robust", exclude=None):
    """First hit id (-1: none) and t of each half-line, t in (0, t_far], under
    the hit rule `rule`; exclude as for ``query``."""
    V = _c(V, np.float32); F = _c(F, np.int32); P = _c(P, np.float64); D = _c(D, np.float64)
    n = P.shape[0]
    ids = np.zeros(n, np.int32); t = np.zeros(n)
    ex = _exclude(exclude, n)
    fn = "orc_first_hit_brute" if method == "brute" else "orc_first_hit_bvh"
    _call(fn, _p(V), _p(F), C.c_int64(F.shape[0]), C.c_int64(n), _p(P), _p(D), C.c_double(t_far),
          _rule(rule), _p(ex), _p(ids), _p(t))
    return ids, t


def visibility(V, F, eyes, target, tan_half, res, t_far, method="bvh"):
    """Per-ray first hits [n_views, res, res] and the per-face visibility mask."""
    P, D = camera_rays(eyes, target, tan_half, res)
    ids, t = first_hit(V, F, P, D, t_far, method)
    vis = np.zeros(np.asarray(F).shape[0], bool)
    vis[ids[ids >= 0]] = True
    return ids.reshape(-1, res, res), t.reshape(-1, res, res), vis


def flood_fill(V, F, seed):
    """Exterior mask: the seeds and every face connected to one through shared
    edges whose two faces' normals agree in direction."""
    V = _c(V, np.float32); F = _c(F, np.int32); sd = _c(np.asarray(seed, bool), np.uint8)
    ext = np.zeros(F.shape[0], np.uint8)
    _call("orc_flood_fill", _p(V), C.c_int64(V.shape[0]), _p(F), C.c_int64(F.shape[0]), _p(sd), _p(ext))
    return ext.astype(bool)


# ---------------------------------------------------------------------------
# Backprojection precompute (Sec. 7.4, TextureGen Postprocessing)
# ---------------------------------------------------------------------------

@dataclass
class ViewMaps:
    texels: np.ndarray     # covered texels (row-major index)
    P: np.ndarray          # [n, 3] surface points
    N: np.ndarray          # [n, 3] unit smooth normals
    ok: np.ndarray         # [n] normal defined
    ray_t: np.ndarray      # [K, res_img, res_img] first-hit t of the depth rays (0: none)
    ray_id: np.ndarray     # [K, res_img, res_img] first-hit face (-1: none)
    uv: np.ndarray         # [K, n, 2] image coordinates (-1, -1 outside)
    inc: np.ndarray        # [K, n] incidence after the visibility test


def view_maps(V, F, UV, res, eyes, target, tan_half, img_res, t_far, tol, method="bvh") -> ViewMaps:
    """Per covered texel of the res^2 atlas and per view: image coordinates,
    incidence max(0, n . d_k) and the depth-buffer visibility test (readings
    in oracle.c)."""
    face, bary = raster(UV, res)
    vn, _ = lo_normals(V, F)
    texels = np.nonzero(face >= 0)[0]
    P, N, ok = rays(V, F, vn, face[texels], bary[texels])
    eyes = _c(eyes, np.float32).reshape(-1, 3)
    Pc, Dc = camera_rays(eyes, target, tan_half, img_res)
    ids, t = first_hit(V, F, Pc, Dc, t_far, method)
    K, n = eyes.shape[0], texels.size
    uv = np.zeros((K, n, 2)); inc = np.zeros((K, n))
    tg = _c(np.asarray(target, np.float32), np.float64).reshape(3)
    okc = _c(ok, np.uint8)
    _call("orc_view_maps", _p(P), _p(N), _p(okc), C.c_int64(n), _p(eyes), C.c_int32(K), _p(tg),
          C.c_double(tan_half), C.c_int32(img_res), _p(t), C.c_double(tol), _p(uv), _p(inc))
    return ViewMaps(texels, P, N, ok, t.reshape(K, img_res, img_res), ids.reshape(K, img_res, img_res), uv, inc)



# ------------------------------------------------------------ simplification

def qem_quadrics(V, F):
    """Per-vertex quadrics [nv, 10] (q00 q01 q02 q03 q11 q12 q13 q22 q23 q33)."""
    V = _c(V, np.float32); F = _c(F, np.int32)
    Q = np.zeros((V.shape[0], 10))
    _call("orc_qem_quadrics", _p(V), C.c_int64(V.shape[0]), _p(F), C.c_int64(F.shape[0]), _p(Q))
    return Q


@dataclass
class QemEdges:
    edges: np.ndarray    # [ne, 2] int32, v0 < v1, in (v0, v1) order
    valid: np.ndarray    # [ne] bool
    faces: np.ndarray    # [ne] faces of the edge (= faces a collapse removes)
    cost: np.ndarray     # [ne] float64
    p: np.ndarray        # [ne, 3] float64 placement


def qem_edges(V, F, Q=None, midpoint=False):
    """Every edge of the mesh (FP64 positions; vertex quadrics Q, default from
    the faces) with its collapse evaluated (placement, cost, validity)."""
    V = _c(V, np.float64); F = _c(F, np.int32)
    Qc = None if Q is None else _c(Q, np.float64)
    cap = 3 * F.shape[0] + 16
    E = np.zeros((cap, 2), np.int32); ok = np.zeros(cap, np.uint8); nf = np.zeros(cap, np.int32)
    cost = np.zeros(cap); P = np.zeros((cap, 3)); n = np.zeros(1, np.int64)
    _call("orc_qem_edges", _p(V), C.c_int64(V.shape[0]), _p(F), C.c_int64(F.shape[0]), _p(Qc),
          C.c_int32(int(midpoint)), C.c_int64(cap), _p(E), _p(ok), _p(nf), _p(cost), _p(P), _p(n))
    k = int(n[0])
    return QemEdges(E[:k], ok[:k].astype(bool), nf[:k], cost[:k], P[:k])


@dataclass
class QemResult:
    V: np.ndarray        # [nv', 3] float64
    F: np.ndarray        # [nf', 3] int32
    rounds: int          # rounds run (round schedule) or collapses (greedy)
    stats: np.ndarray    # [rounds, 4]: edges, valid edges, collapses, faces after (round schedule)


def qem_simplify(V, F, target, method="rounds", rho=0.25, max_rounds=1000, midpoint=False) -> QemResult:
    """Simplify to `target` faces: the parallel round schedule or the serial
    greedy order (``qem.c`` states both)."""
    V = _c(V, np.float32); F = _c(F, np.int32)
    nv, nf = V.shape[0], F.shape[0]
    Vo = np.zeros((max(nv, 1), 3)); Fo = np.zeros((max(nf, 1), 3), np.int32); cnt = np.zeros(2, np.int64)
    if method == "rounds":
        st = np.zeros((max(max_rounds, 1), 4), np.int64); nr = np.zeros(1, np.int32)
        _call("orc_qem_rounds", _p(V), C.c_int64(nv), _p(F), C.c_int64(nf), C.c_int64(target), C.c_double(rho),
              C.c_int32(max_rounds), C.c_int32(int(midpoint)), _p(Vo), _p(Fo), _p(cnt), _p(st), _p(nr))
        r = int(nr[0])
        return QemResult(Vo[:cnt[0]], Fo[:cnt[1]], r, st[:r])
    if method == "greedy":
        done = np.zeros(1, np.int64)
        _call("orc_qem_greedy", _p(V), C.c_int64(nv), _p(F), C.c_int64(nf), C.c_int64(target),
              C.c_int32(int(midpoint)), _p(Vo), _p(Fo), _p(cnt), _p(done))
        return QemResult(Vo[:cnt[0]], Fo[:cnt[1]], int(done[0]), np.zeros((0, 4), np.int64))
    raise ValueError(method)


def sample_surface(V, F, n, seed):
    """n points uniformly by area on the mesh (seeded)."""
    V = np.asarray(V, np.float64); F = np.asarray(F, np.int64)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    rng = np.random.default_rng(seed)
    f = rng.choice(F.shape[0], size=n, p=area / area.sum())
    r1, r2 = rng.random(n), rng.random(n)
    s = np.sqrt(r1)
    return (1 - s)[:, None] * a[f] + (s * (1 - r2))[:, None] * b[f] + (s * r2)[:, None] * c[f]


def mesh_distance(VA, FA, VB, FB, n=4000, seed=0):
    """Two-sided sampled surface distance: (Chamfer = mean of the two mean
    point-to-surface distances, Hausdorff = the larger maximum)."""
    out = []
    both = np.concatenate([np.asarray(VA, np.float64), np.asarray(VB, np.float64)])
    reach = 2.0 * float(np.linalg.norm(both.max(0) - both.min(0)))   # beyond any distance between them
    for (V1, F1, V2, F2, sd) in ((VA, FA, VB, FB, seed), (VB, FB, VA, FA, seed + 1)):
        P = sample_surface(V1, F1, n, sd)
        ids, d, _ = closest(np.asarray(V2, np.float32), F2, P, reach, method="bvh")
        assert (ids >= 0).all()
        out.append(d)
    return 0.5 * (out[0].mean() + out[1].mean()), max(out[0].max(), out[1].max())
