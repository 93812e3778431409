"""Quadrature rules used by the oracle (test infrastructure; see oracle/__init__.py).

The paper does not fix its quadrature.  The reading used here: a 7-point degree-5 rule on each
triangle of a disjoint pair (49 kernel evaluations), Gauss-Legendre products inside the
Duffy-regularised rules for pairs that share a vertex, an edge or the whole triangle.
"""
from __future__ import annotations

import math

import numpy as np


def triangle7():
    """Radon's 7-point rule (degree 5) on a triangle, barycentric points and weights summing to 1.

    Points: the centroid and two orbits (1-2a, a, a) with a = (6 -+ sqrt 15)/21.
    Weights: 9/40 and (155 -+ sqrt 15)/1200.  Exactness on all monomials of degree <= 5 is
    pinned in tests/test_oracle_quadrature.py against the closed form i! j! / (i+j+2)!.
    """
    s15 = math.sqrt(15.0)
    a1 = (6.0 - s15) / 21.0
    a2 = (6.0 + s15) / 21.0
    w1 = (155.0 - s15) / 1200.0
    w2 = (155.0 + s15) / 1200.0
    bary = [(1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0)]
    wts = [9.0 / 40.0]
    for a, w in ((a1, w1), (a2, w2)):
        b = 1.0 - 2.0 * a
        bary += [(b, a, a), (a, b, a), (a, a, b)]
        wts += [w, w, w]
    return np.array(bary), np.array(wts)


def gauss_legendre01(n: int):
    """n-point Gauss-Legendre nodes and weights on [0, 1] (numpy's leggauss, mapped)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w
