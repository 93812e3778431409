"""Pins of the oracle's double-layer potential (Lemma repDL, eq. formulaDL); CPU only."""
import math

import numpy as np
from scipy import integrate

from paper_2310_09204_amd import meshes
from oracle.potential import double_layer, solid_angle

X = np.array([[0.5, 0.5, 0.5], [0.3, 0.7, -0.4], [1.5, 0.2, 0.3], [0.5, 0.5, 2.0], [0.1, 0.9, 0.25]])


def test_constant_jump_is_the_solid_angle():
    # [u] = 1 on a flat screen: U(x) = solid angle / (4 pi), positive on the side n_T points to;
    # the 7-point rule converges like h^6
    errs = []
    for n in (8, 16, 32):
        m = meshes.unit_square(n)
        U = double_layer(m.vertices, m.triangles, np.ones((m.nt, 3)), X)
        ref = solid_angle(m.vertices, m.triangles, X) / (4 * math.pi)
        errs.append(np.abs(U - ref).max())
    assert abs(ref[0] - 1.0 / 6.0) < 1e-14          # a face of a cube seen from its centre
    assert errs[1] < errs[0] / 30 and errs[2] < errs[1] / 30
    assert errs[2] < 3e-11


def test_linear_jump_against_adaptive_quadrature():
    # [u](y) = 0.3 + 0.8 y1 - 0.5 y2 on the unit square (normal +z), interpolated exactly by the
    # piecewise-linear jump; reference: adaptive quadrature of z f(y) / (4 pi |x - y|^3)
    f = lambda y1, y2: 0.3 + 0.8 * y1 - 0.5 * y2
    m = meshes.unit_square(32)
    jump = f(m.vertices[m.triangles][..., 0], m.vertices[m.triangles][..., 1])
    U = double_layer(m.vertices, m.triangles, jump, X[:3])
    for i, x in enumerate(X[:3]):
        g = lambda y2, y1: x[2] * f(y1, y2) / (4 * math.pi * ((x[0] - y1) ** 2 + (x[1] - y2) ** 2 + x[2] ** 2) ** 1.5)
        ref, _ = integrate.dblquad(g, 0.0, 1.0, 0.0, 1.0, epsabs=1e-14, epsrel=1e-13)
        assert abs(U[i] - ref) < 1e-11, (i, U[i], ref)


def test_rigid_motion_and_columns():
    m = meshes.book(4)
    rng = np.random.default_rng(3)
    jump = rng.standard_normal((2, m.nt, 3))
    Xb = np.array([[0.7, 0.4, 0.9], [-0.8, 0.2, -0.5]])
    U = double_layer(m.vertices, m.triangles, jump, Xb)
    th = 0.7
    Q = np.array([[math.cos(th), -math.sin(th), 0.0], [math.sin(th), math.cos(th), 0.0], [0.0, 0.0, 1.0]])
    s = np.array([0.3, -1.2, 2.0])
    U2 = double_layer(m.vertices @ Q.T + s, m.triangles, jump, Xb @ Q.T + s)
    assert np.abs(U2 - U).max() < 1e-13 * np.abs(U).max()
    # columns are independent, and the map is linear in the jump
    U0 = double_layer(m.vertices, m.triangles, jump[0], Xb)
    assert np.abs(U0 - U[0]).max() < 1e-15 * np.abs(U).max()
    Us = double_layer(m.vertices, m.triangles, jump[0] + 2 * jump[1], Xb)
    assert np.abs(Us - (U[0] + 2 * U[1])).max() < 1e-14 * np.abs(Us).max()


def _disk_axis_exact(z):
    # U(0, 0, z) = (z / 2) int_0^1 [u](r) r / (r^2 + z^2)^(3/2) dr for the exact jump of the flat
    # unit disk with g = e_z, [u](r) = -(4/pi) sqrt(1 - r^2)
    f = lambda r: -(4.0 / math.pi) * math.sqrt(1.0 - r * r) * r / (r * r + z * z) ** 1.5
    return 0.5 * z * integrate.quad(f, 0.0, 1.0, epsabs=1e-14, epsrel=1e-13)[0]


def test_disk_solution_on_the_axis():
    # the potential of the discrete disk solution converges to the exact one at first order in h
    # (the jump has a square-root edge singularity), and is odd in z
    from oracle.assemble import assemble, rhs
    from oracle.solve import cholesky_solve
    from oracle.topology import Topology
    zs = np.array([0.5, 1.0, 2.0, -1.0])
    exact = np.array([_disk_axis_exact(z) for z in zs])
    X = np.stack([np.zeros_like(zs), np.zeros_like(zs), zs], axis=1)
    errs = []
    for rings in (4, 8, 12):
        m = meshes.disk(rings)
        t = Topology(m.vertices, m.triangles)
        W = assemble(m.vertices, m.triangles, t, 10)
        phi = cholesky_solve(W, rhs(t, (0.0, 0.0, 1.0))[:, 0])
        U = double_layer(m.vertices, m.triangles, t.jump_values(phi), X)
        assert abs(U[1] + U[3]) < 1e-14
        errs.append(np.abs(U - exact).max() / np.abs(exact).max())
    rate = math.log(errs[0] / errs[2]) / math.log(12 / 4)
    assert 0.8 < rate < 1.4 and errs[2] < 0.02, (errs, rate)
