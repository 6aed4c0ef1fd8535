"""GPU-vs-oracle comparator for the normal bake.

The oracle bakes under two hit rules (oracle.c states both): the plain
definition of the nearest hit ("plain": the line meets the triangle, winner
min (|t|, index)) and the convention the GPU library implements ("robust": a
relative edge tolerance EDGE_EPS on the barycentric weights and a distance
quantum w = max_dist 2^-20, winner min (floor(|t| / w), index)).

``compare`` checks the GPU against the robust rule:
  1. coverage (uncovered status) is bit-identical, and so is the unreliable
     status;
  2. on covered, reliable texels the hit ids agree on at least 99.9 % of them;
  3. every id disagreement is explained by FP32 noise at the rule's
     boundaries, checked in FP64 along the oracle's ray (``fence_ties``): the
     GPU's answer must be the rule's answer over a candidate set that differs
     from the oracle's only by triangles within the FP32 noise bound of the
     tolerance boundary or of the range ends, with distances equal within two
     quanta.  In particular a GPU miss, or a farther GPU hit, is accepted only
     where the oracle's own pick could be lost to the noise AND the GPU matches
     the oracle's runner-up with that pick excluded -- a ray leaking through a
     shared edge of a closed mesh fails, because the runner-up is the other
     face of the edge;
  4. on same-id texels the angle between the tangent-space vectors is at most
     0.05 degrees;
  5. after dilation, uncovered texels agree within 0.05 degrees except next to
     a tie.

``compare_plain`` measures the GPU against the plain rule and reports it:
the agreement rate, and every disagreement must be a tie in the sense of
the bake's accuracy bar: |t| within 1e-6 max_dist of the plain nearest hit,
the GPU's triangle crossed within 32 FP32 ulps of the crossing point, and the
baked normals within 0.05 degrees (a GPU miss only at the range end).

FP32 noise bound (``bake_ray_noise``): the GPU forms a texel's ray origin as
p = b0 V0 + b1 V1 + b2 V2 with b1 = E1/S and b2 = E2/S rounded from exact
integers (each within 3u relative, u = 2^-24) and b0 = 1 - b1 - b2 (within
5u absolute), then a three-term sum (2u): per coordinate |p32 - p| <= 10 u R
with R the largest low-poly coordinate, so |p32 - p| <= 10 sqrt(3) u R.  The
direction d = normalise(sum b_k n_k) carries the rounding of the low-poly
normals and of the sum, within 24 u radians, which moves the crossing by at
most 24 u |t|.  The watertight test's own arithmetic (vertex - origin
differences, the shear, products of sheared coordinates) adds 8 u (|t| +
h_max) in position and 16 u in the weights.  A weight of triangle g moves by
at most (position error) / h_min(g), h_min its smallest altitude: that is the
slack of g on that ray.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ANGLE_TOL_DEG = 0.05
AGREE_MIN = 0.999
TIE_REL = 1e-6
EDGE_EPS = 1.0 / 16384.0  # the robust rule's edge tolerance (barycentric units)
U32 = 2.0 ** -24          # FP32 unit roundoff
MAX_LEVELS = 4            # runner-up levels the fence check may walk


def angle_deg(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    c = np.linalg.norm(np.cross(a, b), axis=-1)
    d = np.einsum("...i,...i->...", a, b)
    return np.degrees(np.arctan2(c, d))


def ulp32(x):
    """Spacing of FP32 numbers at |x| (normal range)."""
    x = np.maximum(np.abs(np.asarray(x, np.float64)), 2.0 ** -126)
    return np.ldexp(1.0, np.floor(np.log2(x)).astype(np.int64) - 23)


def altitudes(V, F, g):
    """Smallest and largest altitude of triangles g (ids >= 0)."""
    V = np.asarray(V, np.float64)
    T = V[np.asarray(F)[np.asarray(g, np.int64)]]
    e = np.stack([T[:, 2] - T[:, 1], T[:, 0] - T[:, 2], T[:, 1] - T[:, 0]], 1)
    le = np.linalg.norm(e, axis=2)
    area2 = np.linalg.norm(np.cross(e[:, 0], e[:, 1]), axis=1)
    h = area2[:, None] / np.maximum(le, 1e-300)
    return h.min(1), h.max(1)


def bake_ray_noise(asset) -> float:
    """Bound on the distance between the GPU's FP32 texel ray and the oracle's
    FP64 ray at |t| = 0 (module docstring)."""
    R = float(np.abs(np.asarray(asset.lo_V, np.float64)).max()) if np.asarray(asset.lo_V).size else 0.0
    return 10.0 * math.sqrt(3.0) * U32 * R


def weight_slack(eps0, t, hmin, hmax, dir_err=24.0 * U32):
    """FP32 noise bound on a barycentric weight of a triangle crossed at t by a
    ray whose origin is within eps0 and direction within dir_err radians."""
    pos = eps0 + dir_err * np.abs(t) + 8.0 * U32 * (np.abs(t) + hmax)
    return pos / np.maximum(hmin, 1e-300) + 16.0 * U32


@dataclass
class FenceResult:
    ok: np.ndarray        # per ray: the disagreement is explained
    level: np.ndarray     # runner-up levels walked (0: the oracle's own pick)
    tie_t: np.ndarray     # accepted as a distance tie (same bin within 2 quanta)
    added: np.ndarray     # accepted as a triangle the GPU admitted within noise
    dropped: np.ndarray   # accepted after dropping fence picks of the oracle


def fence_ties(oracle, V, F, P, D, g, o, o_t, eps0, lim, one_sided=False, method="brute",
               dir_err=24.0 * U32):
    """Is each GPU answer g (-1 miss) the robust rule's answer over a candidate
    set that differs from the oracle's (answer o, distance o_t) only within the
    FP32 noise of the rule's boundaries?  P, D: the oracle's FP64 rays; eps0:
    origin noise bound per ray (scalar or [n]); lim: max_dist (two-sided
    |t| <= lim) or t_far (one-sided 0 < t <= lim)."""
    n = len(g)
    g = np.asarray(g, np.int64)
    ref = np.asarray(o, np.int64).copy()
    ref_t = np.asarray(o_t, np.float64).copy()
    eps0 = np.broadcast_to(np.asarray(eps0, np.float64), (n,)).copy()
    w = lim * 2.0 ** -20
    res = FenceResult(np.zeros(n, bool), np.zeros(n, np.int64), np.zeros(n, bool), np.zeros(n, bool),
                      np.zeros(n, bool))
    if n == 0:
        return res
    P = np.asarray(P, np.float64)
    D = np.asarray(D, np.float64)
    dist = (lambda x: x) if one_sided else np.abs

    def in_range(t, slack_t):
        if one_sided:
            return (t > -slack_t) & (t <= lim * (1 + TIE_REL) + slack_t)
        return np.abs(t) <= lim * (1 + TIE_REL) + slack_t

    def probe(ids):
        """(t, smallest weight, slack of that weight, t noise) of triangle ids."""
        t = np.full(n, np.nan); bm = np.full(n, -np.inf); sl = np.zeros(n); tn = np.zeros(n)
        j = np.nonzero(ids >= 0)[0]
        if j.size:
            tj, _, bj = oracle.plane_check(V, F, P[j], D[j], ids[j].astype(np.int32))
            hmin, hmax = altitudes(V, F, ids[j])
            t[j] = tj
            bm[j] = bj
            sl[j] = weight_slack(eps0[j], tj, hmin, hmax, dir_err)
            tn[j] = 4.0 * U32 * np.abs(tj)
        return t, bm, sl, tn

    tg, bmg, slg, tng = probe(g)
    cand_g = (g >= 0) & (bmg >= -EDGE_EPS - slg) & in_range(tg, tng)
    # a candidate the oracle itself rejected (outside the tolerance or the
    # range in FP64): only such a triangle can beat the oracle's pick
    admitted_g = cand_g & ((bmg < -EDGE_EPS) | ~in_range(tg, 0.0))
    excl = np.full((n, MAX_LEVELS), -1, np.int64)
    todo = np.ones(n, bool)
    for level in range(MAX_LEVELS + 1):
        # does the GPU answer match the current reference answer?
        both_miss = (g < 0) & (ref < 0)
        same = (g >= 0) & (g == ref)
        near = cand_g & (ref >= 0) & (np.abs(dist(tg) - dist(ref_t)) <= 2 * w + tng)
        better = admitted_g & ((ref < 0) | (dist(tg) <= dist(ref_t) + 2 * w + tng))
        m = todo & (both_miss | same | near | better)
        res.ok |= m
        res.level[m] = level
        res.tie_t |= m & near & ~same
        res.added |= m & better & ~near & ~same
        res.dropped |= m & (level > 0)
        todo &= ~m
        if not todo.any() or level == MAX_LEVELS:
            break
        # otherwise the oracle's reference pick must be one the GPU could lose
        # to noise: within the slack of the tolerance boundary or of a range end
        tr, bmr, slr, tnr = probe(np.where(todo, ref, -1))
        if one_sided:
            at_end = (tr >= lim * (1 - TIE_REL) - tnr) | (tr <= eps0 + 4 * U32)
        else:
            at_end = np.abs(tr) >= lim * (1 - TIE_REL) - tnr
        droppable = todo & (ref >= 0) & ((bmr < -EDGE_EPS + slr) | at_end)
        todo &= droppable
        if not todo.any():
            break
        j = np.nonzero(todo)[0]
        excl[j, level] = ref[j]
        if one_sided:
            ids, tt = oracle.first_hit(V, F, P[j], D[j], lim, method=method, rule="robust", exclude=excl[j])
        else:
            ids, tt, _ = oracle.query(V, F, P[j], D[j], lim, method=method, rule="robust", exclude=excl[j])
        ref[j] = ids
        ref_t[j] = np.where(ids >= 0, tt, np.nan)
    return res


@dataclass
class Report:
    n_covered: int = 0
    n_compared: int = 0
    agree: float = 1.0
    n_disagree: int = 0
    n_ties: int = 0
    n_tie_t: int = 0
    n_added: int = 0
    n_dropped: int = 0
    max_angle: float = 0.0
    p999_angle: float = 0.0
    mean_angle: float = 0.0
    max_dilated_angle: float = 0.0
    failures: list = field(default_factory=list)

    def ok(self):
        return not self.failures

    def __str__(self):
        return (f"covered={self.n_covered} compared={self.n_compared} agree={self.agree:.6f} "
                f"disagree={self.n_disagree} ties={self.n_ties} (distance {self.n_tie_t}, "
                f"admitted {self.n_added}, runner-up {self.n_dropped}) angle max={self.max_angle:.2e} "
                f"p99.9={self.p999_angle:.2e} mean={self.mean_angle:.2e} "
                f"dilated max={self.max_dilated_angle:.2e} failures={self.failures[:5]}")


def _query_method(asset):
    return "brute" if np.asarray(asset.hi_F).shape[0] <= 200_000 else "bvh"


def compare(oracle, asset, ob, gpu_map: np.ndarray, gpu_hit: np.ndarray, check_dilation=True,
            agree_min=AGREE_MIN) -> Report:
    """ob: oracle Bake under the robust rule (full or sampled); gpu_map
    [res*res,3], gpu_hit [res*res].  agree_min=None leaves the agreement rate
    to the caller (a sample too small to measure a 0.1 % rate: bound the
    number of ties instead)."""
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
    # 3. every disagreement must be explained by the noise at the rule's fences
    if rep.n_disagree:
        idx = np.nonzero(dis)[0]
        gg = np.where(g[idx] >= 0, g[idx], -1)
        fr = fence_ties(oracle, asset.hi_V, asset.hi_F, ob.P[idx], ob.D[idx], gg, oh[idx],
                        np.where(oh[idx] >= 0, ob.t[idx], np.nan), bake_ray_noise(asset), md,
                        method=_query_method(asset))
        ok = fr.ok & (g[idx] >= -1)
        rep.n_ties = int(ok.sum())
        rep.n_tie_t = int((ok & fr.tie_t).sum())
        rep.n_added = int((ok & fr.added).sum())
        rep.n_dropped = int((ok & fr.dropped).sum())
        if not ok.all():
            bad = idx[~ok][:5]
            rep.failures.append(
                f"{int((~ok).sum())} non-tie disagreements, e.g. texels {tex[bad].tolist()} "
                f"gpu {g[bad].tolist()} oracle {ost[bad].tolist()}")
    if agree_min is not None and rep.agree < agree_min:
        rep.failures.append(f"id agreement {rep.agree:.6f} < {agree_min}")
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


@dataclass
class PlainReport:
    n_compared: int = 0
    agree: float = 1.0
    n_disagree: int = 0
    n_ties: int = 0
    max_dt_rel: float = 0.0      # max | |t_g| - tau* | / max_dist over both-hit disagreements
    max_delta_ulp: float = 0.0   # max crossing distance from the GPU's triangle, in FP32 ulps of |q|
    max_angle: float = 0.0       # max angle between the GPU's and the plain oracle's normal there
    failures: list = field(default_factory=list)

    def ok(self):
        return not self.failures

    def __str__(self):
        return (f"plain rule: compared={self.n_compared} agree={self.agree:.6f} disagree={self.n_disagree} "
                f"ties={self.n_ties} max|dt|/max_dist={self.max_dt_rel:.2e} max delta={self.max_delta_ulp:.2f} ulp "
                f"max angle={self.max_angle:.2e} failures={self.failures[:5]}")


def compare_plain(oracle, asset, obp, gpu_map, gpu_hit) -> PlainReport:
    """The GPU against the oracle's plain rule (obp: an oracle Bake with
    rule="plain", full or sampled).  A disagreement is a tie when the GPU's
    triangle g is crossed by the oracle's ray at |t_g| within 1e-6 max_dist of
    the plain nearest |t| (and within the range), the crossing lies within 32
    FP32 ulps of g, and the baked normals agree within 0.05 degrees; a GPU miss
    against a plain hit, or a GPU hit against a plain miss, is a tie only at
    the range end, the latter also where the ray grazes g (crossing within 32
    ulps of g)."""
    rep = PlainReport()
    md = obp.max_dist
    gm = np.asarray(gpu_map, np.float64).reshape(-1, 3)
    gh = np.asarray(gpu_hit).reshape(-1).astype(np.int64)
    tex = obp.texels
    pst = obp.status[tex].astype(np.int64)
    g = gh[tex]
    rel = (pst != -2) & (g != -2)
    rep.n_compared = int(rel.sum())
    if rep.n_compared == 0:
        return rep
    same = rel & (g == pst)
    dis = rel & ~same
    rep.n_disagree = int(dis.sum())
    rep.agree = float(same.sum()) / rep.n_compared
    if not rep.n_disagree:
        return rep
    idx = np.nonzero(dis)[0]
    gg, pp = g[idx], pst[idx]
    tau = np.where(pp >= 0, np.abs(obp.t[idx]), np.inf)
    ok = np.zeros(idx.size, bool)
    end = lambda x: x >= (1 - TIE_REL) * md
    ok[(gg < 0) & (pp >= 0)] = end(tau[(gg < 0) & (pp >= 0)])
    hg = np.nonzero(gg >= 0)[0]
    if hg.size:
        j = idx[hg]
        tg, dl, _ = oracle.plane_check(asset.hi_V, asset.hi_F, obp.P[j], obp.D[j], gg[hg].astype(np.int32))
        q = obp.P[j] + tg[:, None] * obp.D[j]
        dul = dl / ulp32(np.linalg.norm(q, axis=1))
        in_rng = np.abs(tg) <= md * (1 + TIE_REL)
        ang = angle_deg(gm[tex[j]], obp.map_raw[tex[j]])
        both = pp[hg] >= 0
        t_ok = np.where(both, np.abs(np.abs(tg) - tau[hg]) <= TIE_REL * md, True)
        # where both hit, the normals must agree too; where the plain rule
        # misses, a GPU hit is a tie when the ray grazes g (for instance just
        # outside a boundary edge, which the robust rule's tolerance admits)
        # or crosses it at the range end: the plain map holds no normal there
        ang_ok = np.where(both, ang <= ANGLE_TOL_DEG, True)
        ok[hg] = in_rng & (dul <= 32) & t_ok & ang_ok | (~both & end(np.abs(tg)))
        if both.any():
            rep.max_dt_rel = float((np.abs(np.abs(tg[both]) - tau[hg][both]) / md).max())
        rep.max_delta_ulp = float(dul.max())
        rep.max_angle = float(ang.max())
    rep.n_ties = int(ok.sum())
    if not ok.all():
        bad = idx[~ok][:5]
        rep.failures.append(f"{int((~ok).sum())} non-tie disagreements with the plain rule, e.g. texels "
                            f"{tex[bad].tolist()} gpu {g[bad].tolist()} plain {pst[bad].tolist()}")
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


def closest_near_ties(oracle, asset, ob):
    """Per baked texel of a closest-point oracle bake: a near tie (another
    triangle within two quanta plus NOISE_ABS of the winning distance, not an
    exact tie at a shared vertex or edge)."""
    w = ob.max_dist * 2.0 ** -20
    ids = np.where(ob.hit >= 0, ob.hit, -1).astype(np.int32)
    return oracle.closest_near(asset.hi_V, asset.hi_F, ob.P, ids, ob.t, 2 * w + NOISE_ABS)


def compare_closest(oracle, asset, ob, gpu_map, gpu_hit, check_dilation=True, near=None) -> Report:
    """near (optional, [n baked texels]): the oracle's near ties
    (closest_near_ties).  With it, every id disagreement must also be a near
    tie or a range-end miss, i.e. the GPU agrees on every texel that the FP32
    noise of a distance cannot flip: the agreement floor is 1 - (near-tie
    rate)."""
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
        if near is not None:
            end_miss = (gg == -1) & (tau >= md - NOISE_ABS)
            ok &= np.asarray(near)[idx] | end_miss
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


# ---------------------------------------------------------------------------
# first hits of camera rays (hidden-face removal)
# ---------------------------------------------------------------------------
#
# A camera ray leaves an exact float eye position; the GPU forms its direction
# from the view frame in FP32 (forward, right and up vectors, each normalised,
# and the pixel's offsets), within CAMERA_DIR_ERR radians of the FP64 ray.

CAMERA_DIR_ERR = 32.0 * U32


@dataclass
class RayReport:
    n: int = 0
    agree: float = 1.0
    n_disagree: int = 0
    n_ties: int = 0
    tie_faces: set = field(default_factory=set)
    failures: list = field(default_factory=list)

    def ok(self):
        return not self.failures

    def __str__(self):
        return (f"rays {self.n}: agree {self.agree:.6f} disagree {self.n_disagree} ties {self.n_ties} "
                f"failures={self.failures[:5]}")


def check_first_hits(oracle, V, F, P, D, g_ids, o_ids, o_t, t_far, min_agree=AGREE_MIN,
                     method="brute") -> RayReport:
    """GPU first hits (-1: none) against the oracle's (robust rule) on the same
    camera rays P, D (the oracle's FP64 rays): ids agree on >= min_agree of the
    rays, and every disagreement is explained by the FP32 noise at the rule's
    fences (``fence_ties``, one-sided).  tie_faces: the faces either side named
    on a disagreeing ray."""
    g_ids = np.asarray(g_ids).reshape(-1).astype(np.int64)
    o_ids = np.asarray(o_ids).reshape(-1).astype(np.int64)
    o_t = np.asarray(o_t, np.float64).reshape(-1)
    rep = RayReport(n=int(g_ids.size))
    dis = np.nonzero(g_ids != o_ids)[0]
    rep.n_disagree = int(dis.size)
    rep.agree = 1.0 - dis.size / max(g_ids.size, 1)
    if rep.agree < min_agree:
        rep.failures.append(f"ray agreement {rep.agree:.6f} < {min_agree}")
    if dis.size:
        gg = np.where(g_ids[dis] >= 0, g_ids[dis], -1)
        fr = fence_ties(oracle, V, F, np.asarray(P)[dis], np.asarray(D)[dis], gg, o_ids[dis],
                        np.where(o_ids[dis] >= 0, o_t[dis], np.nan), 0.0, t_far, one_sided=True,
                        method=method, dir_err=CAMERA_DIR_ERR)
        rep.n_ties = int(fr.ok.sum())
        if not fr.ok.all():
            bad = dis[~fr.ok][:5]
            rep.failures.append(f"{int((~fr.ok).sum())} non-tie disagreements, e.g. rays {bad.tolist()} "
                                f"gpu {g_ids[bad].tolist()} oracle {o_ids[bad].tolist()}")
        rep.tie_faces = set(int(x) for x in np.concatenate([g_ids[dis], o_ids[dis]]) if x >= 0)
    return rep


def weight_noise(a, hit):
    """Per hit texel, this module's FP32 noise bound on the GPU's hit weights
    (``weight_slack`` for the hit triangle at the crossing distance t), in the
    form oracle.adjoint_at takes as bnoise."""
    hit = np.asarray(hit).reshape(-1)
    eps0 = bake_ray_noise(a)

    def f(tex, t):
        hmin, hmax = altitudes(a.hi_V, a.hi_F, hit[tex])
        return weight_slack(eps0, t, hmin, hmax)
    return f


def compare_grads(name, g_gpu, g_orc, mag, sens=None, say=None):
    """Check a GPU gradient against the FP64 adjoint at the GPU's selection,
    every entry: relative L2 <= 1e-4 and per entry |gpu - adjoint| <= 1e-3
    |adjoint| + 1e-6 max|adjoint| (+ sens, the adjoint's bound of the terms'
    movement under the FP32 weight noise, where given).  mag: the entries'
    summed term magnitudes (reported in units of u).  Returns the relative L2."""
    if say is None:
        def say(*x):
            print(*x, flush=True)
    g_gpu = np.asarray(g_gpu, np.float64)
    err = np.abs(g_gpu - g_orc)
    rel_l2 = np.linalg.norm(g_gpu - g_orc) / max(np.linalg.norm(g_orc), 1e-30)
    tol = 1e-3 * np.abs(g_orc) + 1e-6 * np.abs(g_orc).max()
    plain = float((err / np.maximum(tol, 1e-300)).max()) if err.size else 0.0
    if sens is not None:
        tol = tol + sens
    ratio = err / np.maximum(tol, 1e-300)
    worst = float(ratio.max()) if err.size else 0.0
    in_u = float((err / np.maximum(U32 * mag, 1e-300)).max()) if err.size else 0.0
    k = np.unravel_index(np.argmax(ratio), ratio.shape) if err.size else None
    extra = f", without the weight-noise term {plain:.3f}" if sens is not None else ""
    say(f"[gpu] grad {name}: {g_orc.size} entries, rel L2 {rel_l2:.2e}, worst err/tol {worst:.3f}"
        f" (entry {k}: gpu {g_gpu[k]:.6e} adjoint {g_orc[k]:.6e} magnitude {mag[k]:.3e}){extra},"
        f" max err / (u magnitude) {in_u:.1f}")
    assert rel_l2 <= 1e-4, rel_l2
    assert worst <= 1.0, worst
    return rel_l2
