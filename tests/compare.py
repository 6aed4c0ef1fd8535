"""GPU-vs-oracle comparator for the normal bake.

Parity rules (what "matches the oracle" means):
  1. coverage (uncovered status) is bit-identical, and so is the unreliable
     status;
  2. on covered, reliable texels the hit ids agree on at least 99.9 % of them;
  3. every id disagreement is a tie of the hit rule, checked in FP64 along the
     oracle's ray: the GPU's triangle g must be a candidate within the FP32
     noise of the rule (smallest barycentric weight of its plane crossing >=
     -EDGE_EPS - 1e-4, |t_g| <= max_dist (1 + 1e-6)) and its distance must be
     within two quanta w = max_dist 2^-20 (about 1e-6 max_dist each) of the
     oracle's best |t|; a GPU miss against an oracle hit, or the reverse, is a
     tie only at the range end (|t| within 1e-6 max_dist of max_dist) or at the
     edge-tolerance boundary (weight within 1e-4 of -EDGE_EPS);
  4. on same-id texels the angle between the tangent-space vectors is at most
     0.05 degrees;
  5. after dilation, uncovered texels agree within 0.05 degrees except next to
     a tie.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

ANGLE_TOL_DEG = 0.05
AGREE_MIN = 0.999
TIE_REL = 1e-6
EDGE_EPS = 1.0 / 16384.0  # the hit rule's edge tolerance (barycentric units)
BARY_SLACK = 1e-4         # FP32 noise allowance on barycentric weights


def angle_deg(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    c = np.linalg.norm(np.cross(a, b), axis=-1)
    d = np.einsum("...i,...i->...", a, b)
    return np.degrees(np.arctan2(c, d))


@dataclass
class Report:
    n_covered: int = 0
    n_compared: int = 0
    agree: float = 1.0
    n_disagree: int = 0
    n_ties: int = 0
    max_angle: float = 0.0
    p999_angle: float = 0.0
    mean_angle: float = 0.0
    max_dilated_angle: float = 0.0
    failures: list = field(default_factory=list)

    def ok(self):
        return not self.failures

    def __str__(self):
        return (f"covered={self.n_covered} compared={self.n_compared} agree={self.agree:.6f} "
                f"disagree={self.n_disagree} ties={self.n_ties} angle max={self.max_angle:.2e} "
                f"p99.9={self.p999_angle:.2e} mean={self.mean_angle:.2e} "
                f"dilated max={self.max_dilated_angle:.2e} failures={self.failures[:5]}")


def compare(oracle, asset, ob, gpu_map: np.ndarray, gpu_hit: np.ndarray, check_dilation=True) -> Report:
    """ob: oracle Bake (full or sampled); gpu_map [res*res,3], gpu_hit [res*res]."""
    rep = Report()
    res, md = ob.res, ob.max_dist
    gm = np.asarray(gpu_map, np.float64).reshape(-1, 3)
    gh = np.asarray(gpu_hit).reshape(-1).astype(np.int64)
    cov = ob.face >= 0
    rep.n_covered = int(cov.sum())
    # 1. coverage
    if not np.array_equal(gh == -3, ~cov):
        bad = np.nonzero((gh == -3) != ~cov)[0]
        rep.failures.append(f"coverage differs at {bad.size} texels, e.g. {bad[:5].tolist()}")
        return rep
    tex = ob.texels
    oh = ob.hit.astype(np.int64)          # oracle query result per baked texel (-2 untraced)
    ost = ob.status[tex].astype(np.int64)  # final oracle status
    g = gh[tex]
    # the unreliable status must match exactly
    if not np.array_equal(g == -2, ost == -2):
        rep.failures.append(f"unreliable status differs at {int(((g == -2) != (ost == -2)).sum())} texels")
    rel = ost != -2
    rep.n_compared = int(rel.sum())
    if rep.n_compared == 0:
        return rep
    same = rel & (g == ost)
    dis = rel & ~same
    rep.n_disagree = int(dis.sum())
    rep.agree = float(same.sum()) / rep.n_compared
    # 3. every disagreement must be a tie
    tie_mask = np.zeros_like(dis)
    if rep.n_disagree:
        w = md * 2.0 ** -20
        idx = np.nonzero(dis)[0]
        o_has = oh[idx] >= 0
        tau = np.where(o_has, np.abs(ob.t[idx]), np.inf)
        gg = g[idx]
        has_g = gg >= 0
        ok = np.zeros(idx.size, bool)
        at_end = lambda x: np.abs(x) >= (1 - TIE_REL) * md
        # is the oracle's own pick at the edge-tolerance boundary?
        o_edge = np.zeros(idx.size, bool)
        if o_has.any():
            j = idx[o_has]
            _, _, bmo = oracle.plane_check(asset.hi_V, asset.hi_F, ob.P[j], ob.D[j], oh[j])
            o_edge[o_has] = np.abs(bmo + EDGE_EPS) <= BARY_SLACK
        # GPU miss against an oracle hit
        gm_ = ~has_g & (gg == -1)
        ok[gm_] = at_end(tau[gm_]) | o_edge[gm_]
        if has_g.any():
            j = idx[has_g]
            tg, _, bm = oracle.plane_check(asset.hi_V, asset.hi_F, ob.P[j], ob.D[j], gg[has_g])
            cand = (bm >= -EDGE_EPS - BARY_SLACK) & (np.abs(tg) <= md * (1 + TIE_REL))
            fin = np.isfinite(tau[has_g])
            t_ok = np.where(fin, np.abs(np.abs(tg) - tau[has_g]) <= 2 * w,
                            at_end(tg) | (np.abs(bm + EDGE_EPS) <= BARY_SLACK))
            ok[has_g] = cand & (t_ok | o_edge[has_g])
        tie_mask[idx] = ok
        rep.n_ties = int(ok.sum())
        if not ok.all():
            bad = idx[~ok][:5]
            rep.failures.append(
                f"{int((~ok).sum())} non-tie disagreements, e.g. texels {tex[bad].tolist()} "
                f"gpu {g[bad].tolist()} oracle {ost[bad].tolist()}")
    if rep.agree < AGREE_MIN:
        rep.failures.append(f"id agreement {rep.agree:.6f} < {AGREE_MIN}")
    # 4. angles on same-id texels (hits and neutral results alike)
    ang = angle_deg(gm[tex][same], ob.map_raw[tex][same])
    if ang.size:
        rep.max_angle = float(ang.max())
        rep.p999_angle = float(np.quantile(ang, 0.999))
        rep.mean_angle = float(ang.mean())
        if rep.max_angle > ANGLE_TOL_DEG:
            rep.failures.append(f"max angle {rep.max_angle:.4f} deg > {ANGLE_TOL_DEG}")
    # 5. dilated texels (full bakes only)
    if check_dilation and tex.size == rep.n_covered:
        unc = np.nonzero(~cov)[0]
        near_tie = np.zeros(res * res, bool)
        if rep.n_disagree:
            t_ids = tex[dis]
            ii, jj = t_ids // res, t_ids % res
            for di in range(-3, 4):
                for dj in range(-3, 4):
                    a, b = ii + di, jj + dj
                    m = (a >= 0) & (b >= 0) & (a < res) & (b < res)
                    near_tie[a[m] * res + b[m]] = True
        unc = unc[~near_tie[unc]]
        if unc.size:
            angd = angle_deg(gm[unc], ob.map[unc])
            rep.max_dilated_angle = float(angd.max())
            if rep.max_dilated_angle > ANGLE_TOL_DEG:
                rep.failures.append(f"dilated max angle {rep.max_dilated_angle:.4f} deg")
    return rep


# ---------------------------------------------------------------------------
# closest-point query
# ---------------------------------------------------------------------------
#
# The closest point of the high-poly is an argmin over triangles decided in
# FP32 on the GPU and in FP64 in the oracle.  Exact ties (a nearest point on a
# shared edge or vertex) resolve to the lower index on both sides; near ties
# (two triangles whose distances differ by less than the FP32 noise of a
# distance, about 1e-7 for O(1) coordinates) may resolve either way, and both
# answers are correct.  So for this query the comparator checks that every id
# disagreement is such a tie (the GPU's triangle, measured in FP64, is within
# two quanta plus NOISE_ABS of the oracle's minimum, or both sit at the range
# end), and compares the baked normals (0.05 degrees) where the ids agree.  A
# near tie is not always between neighbouring triangles: a texel close to the
# medial axis of the surface is equally far from two distinct surface points,
# whose normals differ.

NOISE_ABS = 1e-6  # FP32 distance noise allowance, absolute (coordinates are O(1))


def compare_closest(oracle, asset, ob, gpu_map, gpu_hit, check_dilation=True) -> Report:
    rep = Report()
    res, md = ob.res, ob.max_dist
    gm = np.asarray(gpu_map, np.float64).reshape(-1, 3)
    gh = np.asarray(gpu_hit).reshape(-1).astype(np.int64)
    cov = ob.face >= 0
    rep.n_covered = int(cov.sum())
    if not np.array_equal(gh == -3, ~cov):
        rep.failures.append("coverage differs")
        return rep
    tex = ob.texels
    oh = ob.hit.astype(np.int64)
    ost = ob.status[tex].astype(np.int64)
    g = gh[tex]
    if not np.array_equal(g == -2, ost == -2):
        rep.failures.append(f"unreliable status differs at {int(((g == -2) != (ost == -2)).sum())} texels")
    rel = ost != -2
    rep.n_compared = int(rel.sum())
    if rep.n_compared == 0:
        return rep
    same = rel & (g == ost)
    dis = rel & ~same
    rep.n_disagree = int(dis.sum())
    rep.agree = float(same.sum()) / rep.n_compared
    w = md * 2.0 ** -20
    if rep.n_disagree:
        idx = np.nonzero(dis)[0]
        tau = np.where(oh[idx] >= 0, ob.t[idx], np.inf)
        gg = g[idx]
        ok = np.zeros(idx.size, bool)
        has_g = gg >= 0
        # GPU miss: the oracle's point sits at the range end
        ok[~has_g] = (gg[~has_g] == -1) & (tau[~has_g] >= md - NOISE_ABS)
        if has_g.any():
            j = idx[has_g]
            dg = oracle.closest_check(asset.hi_V, asset.hi_F, ob.P[j], gg[has_g])
            fin = np.isfinite(tau[has_g])
            within = dg <= md + NOISE_ABS
            t_ok = np.where(fin, np.abs(dg - tau[has_g]) <= 2 * w + NOISE_ABS, dg >= md - NOISE_ABS)
            ok[has_g] = within & t_ok
        rep.n_ties = int(ok.sum())
        if not ok.all():
            bad = idx[~ok][:5]
            rep.failures.append(f"{int((~ok).sum())} non-tie disagreements, e.g. texels {tex[bad].tolist()} "
                                f"gpu {g[bad].tolist()} oracle {ost[bad].tolist()}")
    ang = angle_deg(gm[tex][same], ob.map_raw[tex][same])
    if ang.size:
        rep.max_angle = float(ang.max())
        rep.p999_angle = float(np.quantile(ang, 0.999))
        rep.mean_angle = float(ang.mean())
        if rep.max_angle > ANGLE_TOL_DEG:
            rep.failures.append(f"max angle {rep.max_angle:.4f} deg > {ANGLE_TOL_DEG}")
    if check_dilation and tex.size == rep.n_covered:
        unc = np.nonzero(~cov)[0]
        near = np.zeros(res * res, bool)
        bad_t = tex[dis]
        ii, jj = bad_t // res, bad_t % res
        for di in range(-3, 4):
            for dj in range(-3, 4):
                a, b = ii + di, jj + dj
                m = (a >= 0) & (b >= 0) & (a < res) & (b < res)
                near[a[m] * res + b[m]] = True
        unc = unc[~near[unc]]
        if unc.size:
            angd = angle_deg(gm[unc], ob.map[unc])
            rep.max_dilated_angle = float(angd.max())
            if rep.max_dilated_angle > ANGLE_TOL_DEG:
                rep.failures.append(f"dilated max angle {rep.max_dilated_angle:.4f} deg")
    return rep
