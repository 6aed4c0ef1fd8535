"""Pins of the oracle's frozen-selection forward and of its FP64 adjoint.

The frozen forward is pinned to the oracle bake itself at the unperturbed
inputs; the adjoint is pinned by central finite differences of the frozen
forward (h = 1e-4 on the float32 inputs) and by the closed form of the
high-poly-normal derivative.
"""
import numpy as np
import pytest

from synth import make_config


@pytest.fixture(scope="module")
def setup(oracle_lib):
    oracle = oracle_lib
    a = make_config(1)
    ob = oracle.bake(a)
    # texels whose hit sits at least 1e-3 (barycentric) inside its triangle
    ok = (ob.hit >= 0) & (ob.status[ob.texels] >= 0) & (ob.beta.min(1) >= 1e-3)
    idx = np.nonzero(ok)[0]
    rng = np.random.default_rng(4)
    sel = np.sort(rng.choice(idx, size=64, replace=False))
    tex = ob.texels[sel]
    face = ob.face[tex]
    _, vok = oracle.lo_normals(a.lo_V, a.lo_F)
    _, _, hf, _ = oracle.face_frames(a.lo_V, a.lo_F, a.lo_UV, a.res, vok)
    return a, ob, sel, tex, face, ob.bary[tex], ob.hit[sel], hf[face]


def test_frozen_forward_reproduces_the_bake(oracle_lib, setup):
    a, ob, sel, tex, face, bary, g, hf = setup
    out, tb = oracle_lib.frozen_forward(a, face, bary, g, hf)
    assert np.abs(out - ob.map_raw[tex]).max() < 1e-12
    assert np.abs(tb[:, 0] - ob.t[sel]).max() < 1e-12
    assert np.abs(tb[:, 1:] - ob.beta[sel][:, 1:]).max() < 1e-10


def _fd(oracle, a, face, bary, g, hf, gout, which, idx, h=1e-4):
    """Central difference of L = sum gout . out w.r.t. one float32 input."""
    import copy
    arr = getattr(a, which)
    x0 = arr.reshape(-1)[idx]
    vals = []
    xs = []
    for s in (+1, -1):
        b = copy.copy(a)
        pert = arr.copy()
        pert.reshape(-1)[idx] = np.float32(x0 + s * h)
        xs.append(float(pert.reshape(-1)[idx]))
        setattr(b, which, pert)
        out, _ = oracle.frozen_forward(b, face, bary, g, hf)
        vals.append(np.sum(gout * out))
    return (vals[0] - vals[1]) / (xs[0] - xs[1])


def test_adjoint_matches_finite_differences(oracle_lib, setup):
    a, ob, sel, tex, face, bary, g, hf = setup
    rng = np.random.default_rng(9)
    gout = rng.normal(size=(face.size, 3))
    glo, ghi = oracle_lib.adjoint(a, face, bary, g, hf, gout)
    # every coordinate of the low-poly vertices in the faces' 1-ring closure
    lo_verts = np.unique(a.lo_F[np.isin(a.lo_F, a.lo_F[face]).any(1)])
    checked = 0
    for v in lo_verts:
        for k in range(3):
            fd = _fd(oracle_lib, a, face, bary, g, hf, gout, "lo_V", 3 * v + k)
            an = glo[v, k]
            if abs(an) > 1e-8:
                assert abs(fd - an) <= 1e-4 * abs(an) + 1e-9, (v, k, fd, an)
                checked += 1
    assert checked > 50
    hi_verts = np.unique(a.hi_F[g])
    for v in hi_verts[:40]:
        for k in range(3):
            fd = _fd(oracle_lib, a, face, bary, g, hf, gout, "hi_N", 3 * v + k)
            an = ghi[v, k]
            assert abs(fd - an) <= 1e-4 * abs(an) + 1e-9, (v, k, fd, an)
    # vertices no texel touches get nothing
    untouched = np.setdiff1d(np.arange(a.hi_V.shape[0]), hi_verts)
    assert np.all(ghi[untouched] == 0)


def test_hi_normal_gradient_closed_form(oracle_lib, setup):
    """For one ray: d out / d N_k = beta_k [T'; B'; d] (I - n n^T) / |h|."""
    a, ob, sel, tex, face, bary, g, hf = setup
    r = 5
    gout = np.zeros((1, 3)); gout[0] = [0.3, -0.7, 0.2]
    _, ghi = oracle_lib.adjoint(a, face[r:r + 1], bary[r:r + 1], g[r:r + 1], hf[r:r + 1], gout)
    out, tb = oracle_lib.frozen_forward(a, face[r:r + 1], bary[r:r + 1], g[r:r + 1], hf[r:r + 1])
    beta = np.array([1 - tb[0, 1] - tb[0, 2], tb[0, 1], tb[0, 2]])
    N = a.hi_N[a.hi_F[g[r]]].astype(np.float64)
    h = beta @ N
    n = h / np.linalg.norm(h)
    # frame rows from the oracle's own output: out = F n  =>  F^T out = n
    # (F orthonormal); reconstruct F from the tangent definition
    vn, vok = oracle_lib.lo_normals(a.lo_V, a.lo_F)
    Tf, _, hfs, _ = oracle_lib.face_frames(a.lo_V, a.lo_F, a.lo_UV, a.res, vok)
    b = bary[r]
    m = b @ vn[a.lo_F[face[r]]]
    d = m / np.linalg.norm(m)
    T = Tf[face[r]] - (d @ Tf[face[r]]) * d
    T /= np.linalg.norm(T)
    Bp = hf[r] * np.cross(d, T)
    Fm = np.stack([T, Bp, d])
    assert np.allclose(Fm @ n, out[0], atol=1e-12)
    J = Fm @ (np.eye(3) - np.outer(n, n)) / np.linalg.norm(h)
    for k in range(3):
        exp = beta[k] * (J.T @ gout[0])
        assert np.allclose(ghi[a.hi_F[g[r], k]], exp, atol=1e-12)


def test_bake_adjoint_ignores_non_hits(oracle_lib):
    a = make_config(1)
    ob = oracle_lib.bake(a)
    gm = np.ones((a.res * a.res, 3))
    glo, ghi = oracle_lib.bake_adjoint(a, ob, gm)
    gm2 = gm.copy()
    nonhit = np.ones(a.res * a.res, bool)
    nonhit[ob.texels[(ob.hit >= 0)]] = False
    gm2[nonhit] = 1e6  # non-hit texels are constants: no effect
    glo2, ghi2 = oracle_lib.bake_adjoint(a, ob, gm2)
    assert np.array_equal(glo, glo2) and np.array_equal(ghi, ghi2)


def test_weight_noise_bound_dominates_the_change(oracle_lib, setup):
    """The hi_N sensitivity output (orc_adjoint's bnoise / ghiN_sens) bounds
    the change of dL/dhi_N when the hit weights move.  The weights are moved
    through the geometry: each hit triangle is shifted within its own plane by
    a small random offset (the crossing point, and so beta, moves; the hit
    normals and the upstream gradient do not), and the change of every entry
    must stay within the bound computed with the largest weight change seen
    on that ray.  Brute force over the 64 sampled rays, one ray at a time (so
    a triangle shared by two rays is moved for one of them only)."""
    import copy
    a, ob, sel, tex, face, bary, g, hf = setup
    rng = np.random.default_rng(21)
    gout = rng.normal(size=(face.size, 3))
    worst = 0.0
    for r in range(face.size):
        sl = slice(r, r + 1)
        _, ghi0 = oracle_lib.adjoint(a, face[sl], bary[sl], g[sl], hf[sl], gout[sl])
        _, tb0 = oracle_lib.frozen_forward(a, face[sl], bary[sl], g[sl], hf[sl])
        T = a.hi_V[a.hi_F[g[r]]].astype(np.float64)
        e1, e2 = T[1] - T[0], T[2] - T[0]
        u = e1 / np.linalg.norm(e1)
        w = np.cross(np.cross(e1, e2), u)
        w /= np.linalg.norm(w)
        for _ in range(3):
            # an in-plane shift of about 1e-3 of the triangle's size: the
            # float32 vertices round, so the shift is not exactly in-plane,
            # which only changes beta (and t) a little more
            s = (rng.normal() * u + rng.normal() * w) * 1e-3 * np.linalg.norm(e1)
            b = copy.copy(a)
            hv = a.hi_V.copy()
            for j in a.hi_F[g[r]]:
                hv[j] = (hv[j].astype(np.float64) + s).astype(np.float32)
            b.hi_V = hv
            _, ghi1 = oracle_lib.adjoint(b, face[sl], bary[sl], g[sl], hf[sl], gout[sl])
            _, tb1 = oracle_lib.frozen_forward(b, face[sl], bary[sl], g[sl], hf[sl])
            db = float(np.abs(tb1[0, 1:] - tb0[0, 1:]).max())
            assert db > 0
            _, _, _, _, sens = oracle_lib.adjoint(a, face[sl], bary[sl], g[sl], hf[sl], gout[sl],
                                                  magnitudes=True, bnoise=np.array([db]))
            change = np.abs(ghi1 - ghi0)
            # first order: allow 1 % for the second-order terms at this shift
            assert np.all(change <= 1.01 * sens + 1e-15), (r, change.max(), sens.max())
            touched = np.abs(ghi0).sum(1) > 0
            worst = max(worst, float((change[touched] / np.maximum(sens[touched], 1e-300)).max()))
    # the bound is not vacuous: some entry uses a good part of it
    print(f"largest change / bound: {worst:.3f}")
    assert worst > 0.05, worst
