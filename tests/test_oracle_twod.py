"""Pins of the two-dimensional oracle (segment multiscreens, Section 2 Experiments 1 and 2)."""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_2310_09204_amd import meshes
from oracle.solve import cholesky_solve
from oracle.twod import (Topology2D, assemble, cross_exact, double_layer, pair_integral, rhs)


def test_topology_counts():
    V, S = meshes.plus2d(5)
    t = Topology2D(V, S)
    assert t.q[0] == 4 and t.N == 4 * 4 + 3
    assert sorted(set(t.q[1:].tolist())) == [1, 2]
    V, S = meshes.threefold2d(4)
    t = Topology2D(V, S)
    assert t.q[0] == 3 and t.N == 3 * 3 + 2
    # the jump basis: at an interior vertex of an arm, psi = phi_0 - phi_1 jumps by +1 - (-1) = 2
    # (its traces are +1 on one side and -1 on the other); at the tips nothing
    V, S = meshes.slit2d(3)
    t = Topology2D(V, S)
    assert t.N == 5 and np.all(np.abs(t.c[t.c != 0]) == 2)


def _brute(xa, xb, ya, yb, touching):
    L1 = np.linalg.norm(np.subtract(xb, xa))
    L2 = np.linalg.norm(np.subtract(yb, ya))
    f = lambda u, t: math.log(np.linalg.norm(np.asarray(xa) + t * (np.subtract(xb, xa)) - np.asarray(ya) - u * np.subtract(yb, ya)))
    val, _ = integrate.dblquad(f, 0.0, 1.0, 0.0, 1.0, epsabs=1e-13, epsrel=1e-12)
    return -L1 * L2 * val / (2 * math.pi)


def test_pair_integrals_against_adaptive_quadrature():
    # a segment with itself (closed form), segments with a common end at several angles, and a
    # disjoint pair, against adaptive quadrature of the defining integral
    x0 = np.array([0.2, -0.1])
    same = pair_integral(x0, x0 + [0.3, 0.4], x0, x0 + [0.3, 0.4], "same")
    # L = 0.5: int_0^1 int_0^1 log(L |t - u|) du dt, the inner integral split at its singular point
    inner = lambda t: (integrate.quad(lambda u: math.log(0.5 * (t - u)), 0.0, t, epsabs=1e-15)[0] if t > 0 else 0.0) + \
        (integrate.quad(lambda u: math.log(0.5 * (u - t)), t, 1.0, epsabs=1e-15)[0] if t < 1 else 0.0)
    ref = -integrate.quad(inner, 0.0, 1.0, epsabs=1e-14, limit=200)[0] * 0.25 / (2 * math.pi)
    assert abs(same - ref) < 1e-10 * abs(ref)
    for ang in (90, 120, 180, 270, 30):
        a = math.radians(ang)
        P = np.array([0.1, 0.2])
        xb = P + 0.3 * np.array([1.0, 0.0])
        yb = P + 0.45 * np.array([math.cos(a), math.sin(a)])
        k = pair_integral(P, xb, P, yb, (0, 0))
        assert abs(k - _brute(P, xb, P, yb, True)) < 1e-9 * abs(k), ang
        # the same pair with the ends listed the other way round
        k2 = pair_integral(xb, P, yb, P, (1, 1))
        assert abs(k2 - k) < 1e-13 * abs(k)
    xa, xb, ya, yb = [0, 0], [0.1, 0.0], [0.3, 0.05], [0.35, 0.15]
    assert abs(pair_integral(xa, xb, ya, yb) - _brute(xa, xb, ya, yb, False)) < 1e-11


def _solve(V, S, g):
    t = Topology2D(V, S)
    W = assemble(t)
    L = rhs(t, g)[:, 0]
    return t, W, L, cholesky_solve(W, L)


def test_symmetric_cross_reduces_to_the_slit():
    # Experiment 1's data g = (0, -1/2): reflection x1 -> -x1 maps the vertical arm to itself and
    # flips its normal, so its jump vanishes, and the horizontal arm carries the slit's solution
    n = 8
    tc, Wc, Lc, phic = _solve(*meshes.plus2d(n), (0.0, -0.5))
    assert np.array_equal(Wc, Wc.T) and np.linalg.eigvalsh(Wc)[0] > 0
    jc = tc.jump_values(phic)
    Vc = tc.V
    vert = [s for s in range(tc.ns) if abs(Vc[tc.S[s, 0], 0]) + abs(Vc[tc.S[s, 1], 0]) < 1e-12]
    assert np.abs(jc[vert]).max() < 1e-12 * np.abs(jc).max()
    ts, Ws, Ls, phis = _solve(*meshes.slit2d(n), (0.0, -0.5))
    js = ts.jump_values(phis)
    # match segments by their end points
    key = lambda V, S, s: tuple(np.round(np.sort(V[S[s]][:, 0]), 12))
    mp = {key(ts.V, ts.S, s): s for s in range(ts.ns)}
    for s in range(tc.ns):
        if s in vert:
            continue
        s2 = mp[key(Vc, tc.S, s)]
        a = 0 if Vc[tc.S[s, 0], 0] < Vc[tc.S[s, 1], 0] else 1
        sg = tc.normal[s, 1] * ts.normal[s2, 1]   # the jump is taken towards the segment's normal
        assert abs(sg * jc[s, a] - js[s2, 0]) < 1e-10 and abs(sg * jc[s, 1 - a] - js[s2, 1]) < 1e-10


def test_experiment1_converges():
    # new method on the uniform cross: the discrete l2 error of U_h on a grid around the cross
    # decreases at first order in h, and the jump approaches sqrt(1 - x1^2)
    g = np.linspace(-1.5, 1.5, 31) + 0.0123
    X = np.array([(a, b) for a in g for b in g])
    exact = cross_exact(X)
    errs = []
    for n in (4, 8, 16):
        t, W, L, phi = _solve(*meshes.plus2d(n), (0.0, -0.5))
        U = double_layer(t, t.jump_values(phi), X)
        errs.append(math.sqrt(np.mean((U - exact) ** 2)))
    rate = math.log(errs[0] / errs[2]) / math.log(4.0)
    assert 0.8 < rate < 1.6 and errs[2] < 0.01, (errs, rate)


def test_double_layer_constant_jump_is_the_angle():
    # [u] = 1 on a segment: U(x) = (signed angle subtended at x) / (2 pi), positive on the normal side
    V, S = meshes.slit2d(16)
    t = Topology2D(V, S)
    X = np.array([[0.2, 0.7], [-0.4, -0.3], [1.6, 0.5]])
    U = double_layer(t, np.ones((t.ns, 2)), X)
    ang = np.array([math.atan2(x[1], x[0] - 1.0) - math.atan2(x[1], x[0] + 1.0) for x in X])
    assert np.abs(U - ang / (2 * math.pi)).max() < 1e-9


def test_coarse_prolongation_2d():
    # the fine jumps of a prolongated coarse basis function are the coarse jumps interpolated by the
    # coarse hat functions (taken towards each fine segment's normal); with ratio 1 R_H = identity
    from oracle.twod import coarse_prolongation_2d
    for kind, n, r in (("threefold", 8, 4), ("plus", 6, 2)):
        (V, S), (cV, cS), par = meshes.arms2d_coarse(kind, n, r)
        f, c = Topology2D(V, S), Topology2D(cV, cS)
        R = coarse_prolongation_2d(f, c, par)
        for i in range(c.N):
            Jf = f.jump_values(R[i])
            e = np.zeros(c.N)
            e[i] = 1.0
            Jc = c.jump_values(e)
            for s in range(f.ns):
                C0, C1 = cV[cS[par[s], 0]], cV[cS[par[s], 1]]
                sg = 1.0 if f.tangent[s] @ c.tangent[par[s]] > 0 else -1.0
                for a in range(2):
                    l1 = (V[S[s, a]] - C0) @ (C1 - C0) / ((C1 - C0) @ (C1 - C0))
                    assert abs(Jf[s, a] - sg * ((1 - l1) * Jc[par[s], 0] + l1 * Jc[par[s], 1])) < 1e-12
    (V, S), (cV, cS), par = meshes.arms2d_coarse("threefold", 4, 1)
    R = coarse_prolongation_2d(Topology2D(V, S), Topology2D(cV, cS), par)
    assert np.abs(R - np.eye(R.shape[0])).max() < 1e-14


def test_experiment2_condition_growth():
    # threefold junction, faces = coarse segments: kappa(P_ad W) grows with H/h no faster than
    # (1 + log(H/h))^2 and hardly depends on H at fixed H/h; kappa(W) grows like 1/h
    from oracle.precond import AdditiveSchwarz
    from oracle.solve import spectral_cond
    from oracle.twod import classify_dofs_2d, coarse_prolongation_2d
    k = {}
    for nc in (2, 4):
        for r in (2, 4, 8, 16):
            (V, S), (cV, cS), par = meshes.arms2d_coarse("threefold", nc * r, r)
            f, c = Topology2D(V, S), Topology2D(cV, cS)
            W = assemble(f)
            faces, wb = classify_dofs_2d(f, par)
            assert len(faces) == 3 * nc and len(wb) == 3 * (nc - 1) + 2
            P = AdditiveSchwarz(W, None, face_sets=faces, wb=wb, RH=coarse_prolongation_2d(f, c, par))
            Md = P.dense(f.N)
            k[(nc, r)] = (spectral_cond(W, 0.5 * (Md + Md.T)), spectral_cond(W))
    for nc in (2, 4):
        kp = [k[(nc, r)][0] for r in (2, 4, 8, 16)]
        assert kp[1] <= kp[2] <= kp[3]
        ratio = [kp[i] / (1 + math.log(r)) ** 2 for i, r in enumerate((2, 4, 8, 16))]
        assert max(ratio) < 1.0
    for r in (2, 4, 8, 16):
        assert abs(k[(2, r)][0] - k[(4, r)][0]) < 0.1 * k[(2, r)][0]
    slope = math.log(k[(2, 16)][1] / k[(2, 2)][1]) / math.log(8.0)
    assert 0.7 < slope < 1.2
