"""Pins of the oracle's quadrature tables and element-pair rules (CPU only)."""
import math

import numpy as np
import pytest

import pins
from oracle.assemble import far_rule, near_rule, pair_integrals
from oracle.quadrature import gauss_legendre01, triangle7

FOUR_PI = 4.0 * math.pi


def test_triangle7_exact_to_degree_5():
    bary, w = triangle7()
    assert abs(w.sum() - 1.0) < 1e-15
    # reference simplex {x,y>=0, x+y<=1}: point = (b1, b2), area 1/2
    x, y = bary[:, 1], bary[:, 2]
    for i in range(6):
        for j in range(6 - i):
            q = 0.5 * float(np.dot(w, x ** i * y ** j))
            assert abs(q - pins.simplex_monomial(i, j)) < 1e-15, (i, j)
    # and it is a degree-5 rule, not better: some degree-6 monomial is missed
    errs = [abs(0.5 * float(np.dot(w, x ** i * y ** (6 - i))) - pins.simplex_monomial(i, 6 - i))
            for i in range(7)]
    assert max(errs) > 1e-6


@pytest.mark.parametrize("n", [2, 6, 10, 16])
def test_gauss_legendre_exactness(n):
    x, w = gauss_legendre01(n)
    for k in range(2 * n):
        assert abs(float(np.dot(w, x ** k)) - 1.0 / (k + 1)) < 1e-14
    if n <= 6:
        assert abs(float(np.dot(w, x ** (2 * n))) - 1.0 / (2 * n + 1)) > 1e-12


def _random_pair(rng, kind):
    A, B, C, B2, C2 = (rng.standard_normal(3) for _ in range(5))
    X = np.array([A, B, C])
    if kind == "coincident":
        return X, X
    if kind == "edge":
        return X, np.array([A, B, C2])
    return X, np.array([A, B2, C2])


def _area(X):
    return 0.5 * np.linalg.norm(np.cross(X[1] - X[0], X[2] - X[0]))


@pytest.mark.parametrize("kind", ["coincident", "edge", "vertex"])
def test_duffy_rules_integrate_constant_kernel_to_area_product(kind):
    # kernel 1: the maps must cover R x R exactly once with the right Jacobian
    rng = np.random.default_rng(7)
    for _ in range(5):
        X, Y = _random_pair(rng, kind)
        v = near_rule(kind, X, Y, 4, kernel=1) * FOUR_PI
        assert abs(v - _area(X) * _area(Y)) < 1e-13 * max(1.0, _area(X) * _area(Y))


@pytest.mark.parametrize("kind", ["coincident", "edge", "vertex"])
@pytest.mark.parametrize("kernel", [2, 3])
def test_duffy_rules_match_product_rule_on_polynomial_kernels(kind, kernel):
    # |x-y|^2 and an asymmetric cubic are integrated exactly by the 7x7 product rule, so any
    # wrong, swapped or transposed map in a Duffy rule shows up here
    rng = np.random.default_rng(11)
    for _ in range(5):
        X, Y = _random_pair(rng, kind)
        v = near_rule(kind, X, Y, 6, kernel=kernel)
        ref = far_rule(X, Y, kernel=kernel)
        assert abs(v - ref) < 1e-12 * max(1.0, abs(ref))


def test_coincident_rule_matches_closed_form():
    for T in (np.array([[0., 0, 0], [1, 0, 0], [1, 1, 0]]),
              np.array([[0., 0, 0], [1, 0, 0], [0.5, math.sqrt(3) / 2, 0]]),
              np.array([[0.3, -0.2, 0.1], [1.4, 0.2, 0.5], [0.2, 0.9, -0.4]])):
        exact = pins.coincident_closed_form(T) / FOUR_PI
        assert abs(near_rule("coincident", T, T, 20) - exact) < 1e-12 * exact
        assert abs(near_rule("coincident", T, T, 10) - exact) < 1e-7 * exact


def test_touching_coplanar_rules_match_planar_potential():
    A = np.array([0., 0, 0]); B = np.array([1., 0, 0]); C = np.array([1., 1, 0])
    T = np.array([A, B, C])
    Te = np.array([A, B, [0.2, -0.9, 0.0]])
    Tv = np.array([A, [-1., 0, 0], [-0.6, -1.1, 0]])
    ref_e = pins.coplanar_pair(T, Te, m=10, depth=9) / FOUR_PI
    ref_v = pins.coplanar_pair(T, Tv, m=10, depth=7) / FOUR_PI
    assert abs(near_rule("edge", T, Te, 16) - ref_e) < 1e-9 * ref_e
    assert abs(near_rule("vertex", T, Tv, 16) - ref_v) < 1e-10 * ref_v
    # production order 10: error of the rule itself
    assert abs(near_rule("edge", T, Te, 10) - ref_e) < 1e-7 * ref_e


@pytest.mark.parametrize("angle", [30.0, 90.0, 120.0, 330.0])
def test_junction_pairs_against_subdivision(angle):
    # non-coplanar pairs across a junction edge / vertex: the rule on the parent pair must equal
    # the sum over 16 x 16 child pairs (separated children by a high-order product rule)
    th = math.radians(angle)
    A = np.array([0., 0, 0]); B = np.array([1., 0, 0]); C = np.array([0.6, 0.8, 0.0])
    C2 = np.array([0.4, 0.8 * math.cos(th), 0.8 * math.sin(th)])
    B2 = np.array([-0.2, 0.9 * math.cos(th), 0.9 * math.sin(th)])
    T = np.array([A, B, C])

    def rule16(kind, X, Y):
        return near_rule(kind, X, Y, 16) * FOUR_PI

    for kind, Y in (("edge", np.array([A, B, C2])), ("vertex", np.array([A, B2, C2]))):
        ref = pins.subdivided_pair(T, Y, rule16, levels=2, m=12) / FOUR_PI
        assert abs(near_rule(kind, T, Y, 16) - ref) < 2e-10 * ref, kind
        assert abs(near_rule(kind, T, Y, 10) - ref) < 2e-7 * ref, kind


def test_far_rule_vs_high_order_and_planar_potential():
    T = np.array([[0., 0, 0], [1, 0, 0], [1, 1, 0]])
    Tf = np.array([[3., 0, 0], [4, 0, 0], [4, 1, 0]])
    exact = pins.coplanar_pair(T, Tf, m=10, depth=0) / FOUR_PI
    assert abs(pins.product_rule_pair(T, Tf, 12) / FOUR_PI - exact) < 1e-13
    assert abs(far_rule(T, Tf) - exact) < 1e-7 * exact


def test_pair_integral_invariants():
    rng = np.random.default_rng(3)
    V = rng.standard_normal((6, 3))
    Tr = np.array([[0, 1, 2], [0, 1, 3], [0, 4, 5], [3, 4, 5]], dtype=np.int32)
    pairs = np.array([[i, j] for i in range(4) for j in range(4)], dtype=np.int32)
    I = pair_integrals(V, Tr, pairs, 10).reshape(4, 4)
    assert np.array_equal(I, I.T)
    lam = 1.7
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    V2 = lam * V @ Q.T + rng.standard_normal(3)
    I2 = pair_integrals(V2, Tr, pairs, 10).reshape(4, 4)
    assert np.allclose(I2, lam ** 3 * I, rtol=1e-12, atol=0)


def test_unit_square_total_matches_coulomb_integral():
    from paper_2310_09204_amd import meshes
    from oracle.assemble import pair_matrix
    exact = pins.unit_square_coulomb() / FOUR_PI
    for n, tol in ((4, 3e-7), (8, 1e-7)):
        m = meshes.unit_square(n)
        tot = pair_matrix(m.vertices, m.triangles, 10).sum()
        assert abs(tot - exact) < tol * exact, n
