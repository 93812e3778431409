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
