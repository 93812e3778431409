"""Independent closed forms and brute-force integrators used to pin the oracle (test code only).

Nothing here is used by the oracle or by the GPU path; these routines exist to check the oracle
against mathematics it does not share code with.
"""
from __future__ import annotations

import math

import numpy as np


def simplex_monomial(i: int, j: int) -> float:
    """int over {x,y >= 0, x + y <= 1} of x^i y^j = i! j! / (i + j + 2)!  (Dirichlet integral)."""
    return math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)


def unit_square_coulomb() -> float:
    """int_{[0,1]^2} int_{[0,1]^2} dx dy / |x - y| = 4 ln(1 + sqrt 2) - (4/3)(sqrt 2 - 1)."""
    r2 = math.sqrt(2.0)
    return 4.0 * math.log(1.0 + r2) - (4.0 / 3.0) * (r2 - 1.0)


def planar_potential(P, tri):
    """V(P) = int_T dy / |P - y| for points P in the plane of T (array (m,3)).

    Polar integration about P: T is the signed sum of the triangles (P, a, b) over its oriented
    edges a -> b, and on each one int 1/r dA = int rho(theta) d theta = d [asinh(s_b/d) - asinh(s_a/d)]
    where d is the distance from P to the edge line and s the coordinate along it from the foot of
    the perpendicular.  The signed distance (positive on the inner side) carries the orientation.
    """
    P = np.atleast_2d(P)
    A, B, C = tri
    n = np.cross(B - A, C - A)
    n = n / np.linalg.norm(n)
    out = np.zeros(P.shape[0])
    for a, b in ((A, B), (B, C), (C, A)):
        e = b - a
        L = np.linalg.norm(e)
        e = e / L
        inward = np.cross(n, e)               # points into T for a counter-clockwise T
        d = (P - a) @ inward                  # signed distance, > 0 inside
        sa = (a - P) @ e
        sb = (b - P) @ e
        ad = np.abs(d)
        ok = ad > 1e-300
        val = np.zeros_like(d)
        val[ok] = d[ok] * (np.arcsinh(sb[ok] / ad[ok]) - np.arcsinh(sa[ok] / ad[ok]))
        out += val
    return out


def _collapsed_rule(m):
    x, w = np.polynomial.legendre.leggauss(m)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    # Duffy-collapsed tensor rule on the unit simplex: (u, v) = (x1, x1 x2) ... mapped to (s, t)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    W1, W2 = np.meshgrid(w, w, indexing="ij")
    s = X1 * (1.0 - X2)
    t = X1 * X2
    wt = W1 * W2 * X1
    return np.stack([1.0 - s - t, s, t], axis=-1).reshape(-1, 3), wt.reshape(-1)


def _children(tri):
    A, B, C = tri
    ab, bc, ca = 0.5 * (A + B), 0.5 * (B + C), 0.5 * (C + A)
    return [np.array([A, ab, ca]), np.array([ab, B, bc]), np.array([ca, bc, C]), np.array([ab, bc, ca])]


def _tri_area(t):
    return 0.5 * np.linalg.norm(np.cross(t[1] - t[0], t[2] - t[0]))


def _touch(t1, t2, eps=1e-12):
    """True if the closed triangles share at least one point (vertex of one on the other)."""
    def on_tri(p, t):
        A, B, C = t
        n = np.cross(B - A, C - A)
        if abs(np.dot(p - A, n)) > eps * np.linalg.norm(n):
            return False
        M = np.stack([B - A, C - A], axis=1)
        lam, *_ = np.linalg.lstsq(M, p - A, rcond=None)
        return lam.min() >= -eps and lam.sum() <= 1 + eps
    return any(on_tri(p, t2) for p in t1) or any(on_tri(p, t1) for p in t2) or \
        min(np.linalg.norm(p - q) for p in t1 for q in t2) < eps


def coplanar_pair(T1, T2, m=10, depth=9):
    """int_T1 int_T2 1/|x-y| for coplanar triangles: exact inner potential (planar_potential),
    outer integral by a collapsed Gauss rule on a subdivision of T1 graded toward T2."""
    bary, w = _collapsed_rule(m)
    T1 = np.asarray(T1, dtype=float)
    T2 = np.asarray(T2, dtype=float)
    total = 0.0
    stack = [(T1, 0)]
    while stack:
        t, lev = stack.pop()
        if lev < depth and _touch(t, T2):
            stack.extend((c, lev + 1) for c in _children(t))
            continue
        pts = bary @ t
        total += 2.0 * _tri_area(t) * float(np.dot(w, planar_potential(pts, T2)))
    return total


def coincident_closed_form(T):
    """int_T int_T 1/|x-y|: the difference x^ - y^ of two points of the reference triangle fills a
    hexagon whose cross-sections are homothetic copies of the triangle; integrating the anchor and
    the radius in closed form leaves three segment integrals int_0^1 d eta / |p + eta q|, each in
    closed form with asinh.  Independent of any quadrature."""
    A, B, C = [np.asarray(v, dtype=float) for v in T]
    M = np.stack([B - A, C - B], axis=1)
    verts = [(1.0, 0.0), (1.0, 1.0), (0.0, 1.0), (-1.0, 0.0)]
    acc = 0.0
    for i in range(3):
        p = M @ np.array(verts[i])
        q = M @ (np.array(verts[i + 1]) - np.array(verts[i]))
        a = q @ q
        b = p @ q
        c = p @ p
        disc = math.sqrt(max(a * c - b * b, 1e-300))
        acc += (math.asinh((a + b) / disc) - math.asinh(b / disc)) / math.sqrt(a)
    area = _tri_area(np.array([A, B, C]))
    return 4.0 * area * area * (1.0 / 3.0) * acc


def product_rule_pair(T1, T2, m=12):
    """Collapsed-Gauss m^2 x m^2 product rule for a separated pair (smooth integrand)."""
    bary, w = _collapsed_rule(m)
    X = bary @ np.asarray(T1, dtype=float)
    Y = bary @ np.asarray(T2, dtype=float)
    r = np.linalg.norm(X[:, None, :] - Y[None, :, :], axis=-1)
    return 4.0 * _tri_area(np.asarray(T1)) * _tri_area(np.asarray(T2)) * float(w @ (1.0 / r) @ w)


def subdivided_pair(T1, T2, touching_rule, levels=2, m=12):
    """Brute force: split both triangles into 4^levels children; touching child pairs go to
    touching_rule(kind, X, Y) with shared vertices first, separated ones to product_rule_pair."""
    def split(t, L):
        out = [np.asarray(t, dtype=float)]
        for _ in range(L):
            out = [c for tt in out for c in _children(tt)]
        return out

    c1, c2 = split(T1, levels), split(T2, levels)
    total = 0.0
    for a in c1:
        for b in c2:
            shared = [(i, j) for i in range(3) for j in range(3) if np.linalg.norm(a[i] - b[j]) < 1e-12]
            if len(shared) == 3:
                total += touching_rule("coincident", a, a)
            elif len(shared) == 2:
                (i0, j0), (i1, j1) = shared
                X = np.array([a[i0], a[i1], a[3 - i0 - i1]])
                Y = np.array([b[j0], b[j1], b[3 - j0 - j1]])
                total += touching_rule("edge", X, Y)
            elif len(shared) == 1:
                (i0, j0), = shared
                X = np.array([a[i0], a[(i0 + 1) % 3], a[(i0 + 2) % 3]])
                Y = np.array([b[j0], b[(j0 + 1) % 3], b[(j0 + 2) % 3]])
                total += touching_rule("vertex", X, Y)
            else:
                total += product_rule_pair(a, b, m)
    return total
