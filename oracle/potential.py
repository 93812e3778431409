"""Double-layer potential of a discrete solution at points off the screen (test infrastructure;
see oracle/__init__.py).

Lemma repDL (eq. formulaDL) writes DL u(x) as a sum over the oriented triangles of
n_t . (y - x) / (4 pi |x - y|^3) times the trace of u on that side.  The two sides of a geometric
triangle T carry the normals -n_T (side +) and +n_T (side -) under the build's orientation reading,
so they combine into one integral of the jump [u]_T = gamma_+ u - gamma_- u:

    U(x) = sum_T  int_T  n_T . (x - y) / (4 pi |x - y|^3)  [u]_T(y)  dsigma(y),

with [u]_T linear on T and equal at corner a to jump[T, a] (Topology.jump_values).  The integral is
taken with the 7-point rule on every triangle, which is accurate for targets a few mesh sizes away
from the screen; there is no refinement for targets close to it.

Pins (tests/test_oracle_potential.py): a constant jump against the closed-form solid angle of the
screen, a linear jump against an adaptive quadrature of the exact integrand, and invariance
under a rigid motion of mesh and targets.
"""
from __future__ import annotations

import numpy as np

from .quadrature import triangle7


def double_layer(V, T, jump, X):
    """U[c, i] for the jump values jump[c, t, a] (or jump[t, a] for one column) at targets X[i]."""
    V = np.asarray(V, dtype=np.float64)
    T = np.asarray(T)
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    J = np.asarray(jump, dtype=np.float64)
    single = J.ndim == 2
    if single:
        J = J[None]
    bary, w = triangle7()
    U = np.zeros((J.shape[0], X.shape[0]))
    for t in range(T.shape[0]):
        x0, x1, x2 = V[T[t, 0]], V[T[t, 1]], V[T[t, 2]]
        cr = np.cross(x1 - x0, x2 - x0)
        area = 0.5 * np.linalg.norm(cr)
        n = cr / (2.0 * area)
        Y = bary @ np.stack([x0, x1, x2])            # 7 Gauss points
        dens = J[:, t, :] @ bary.T                    # [u]_T at the points, per column
        d = X[:, None, :] - Y[None, :, :]             # targets x points x 3
        r = np.sqrt(np.einsum("ipk,ipk->ip", d, d))
        kern = (d @ n) / (4.0 * np.pi * r ** 3)       # targets x points
        U += dens @ (area * w[:, None] * kern.T)
    return U[0] if single else U


def solid_angle(V, T, X):
    """Signed solid angle of the triangles' union seen from X (Van Oosterom-Strackee), positive on
    the side the normals n_T point to."""
    V = np.asarray(V, dtype=np.float64)
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    out = np.zeros(X.shape[0])
    for t in range(len(T)):
        R = [X - V[T[t, a]] for a in range(3)]
        r = [np.linalg.norm(Ra, axis=1) for Ra in R]
        num = np.einsum("ik,ik->i", R[0], np.cross(R[1], R[2]))
        den = (r[0] * r[1] * r[2] + np.einsum("ik,ik->i", R[0], R[1]) * r[2]
               + np.einsum("ik,ik->i", R[0], R[2]) * r[1] + np.einsum("ik,ik->i", R[1], R[2]) * r[0])
        out += 2.0 * np.arctan2(num, den)
    return out
