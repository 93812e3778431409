"""Two-dimensional variant of the method: multiscreens made of line segments in the plane (test
infrastructure; see oracle/__init__.py).

Section 2 (Experiments 1 and 2) runs the same Galerkin method on segment meshes, where the
fundamental solution is -log|x - y| / (2 pi) and the surface curl of a jump is its derivative along
the segment.  Everything mirrors the three-dimensional construction:

  * sectors at a vertex are the angular regions between its segments (q = number of segments; a
    segment end that no other segment meets has q = 1 and no dof);
  * dofs (v, j), j < q - 1, with the jump basis psi_{v,j} = phi_{v,j} - phi_{v,q-1} and the jump
    coefficients c_{s,a,d} = s_+ - s_- at end a of segment s (side + is the side the normal
    n_s = rot90(tau_s) points to, side - the other);
  * W_{dd'} = sum_{s,s'} D_{s,d} D_{s',d'} K(s,s'), with D_{s,d} = (c_{s,1,d} - c_{s,0,d}) / |s| the
    derivative of the jump along s and K(s,s') = -1/(2 pi) int_s int_s' log|x - y|;
  * L_d = -sum_s (g . n_s) |s| / 2 (c_{s,0,d} + c_{s,1,d}) for constant g (the outward-normal
    reading of the three-dimensional right-hand side);
  * U_h(x) = sum_s int_s n_s . (x - y) / (2 pi |x - y|^2) [u]_s(y) dy.

Quadrature (the build's reading, the paper fixes none): 8-point Gauss-Legendre on both segments of
a disjoint pair; the closed form L^2 (log L - 3/2) for a segment with itself; for two segments with
a common end, the split of the square of parameters along its diagonal with the singular factor
integrated exactly, which leaves one regular integral of a logarithm of a quadratic per half (in
closed form).

Experiment 1 (plus-shaped cross) has the exact solution U = Re(-1 / (2 i w)), z = (w + 1/w)/2, whose
Neumann data on the cross equal those of the constant field g = (0, -1/2): its jump is
sqrt(1 - x_1^2) across the horizontal arm and zero across the vertical one.
"""
from __future__ import annotations

import math
from collections import defaultdict

import numpy as np
from .quadrature import gauss_legendre01


class MeshError2D(ValueError):
    pass


class Topology2D:
    """Sectors, dofs and jump coefficients of a segment mesh V (nv x 2), S (ns x 2)."""

    def __init__(self, V, S):
        V = np.asarray(V, dtype=np.float64)
        S = np.asarray(S, dtype=np.int64)
        self.V, self.S = V, S
        ns, nv = S.shape[0], V.shape[0]
        self.ns, self.nv = ns, nv
        d = V[S[:, 1]] - V[S[:, 0]]
        L = np.linalg.norm(d, axis=1)
        if np.any(L <= 0.0):
            raise MeshError2D("degenerate segment")
        if len({tuple(sorted(s)) for s in S.tolist()}) != ns:
            raise MeshError2D("repeated segment")
        self.length = L
        self.tangent = d / L[:, None]
        self.normal = np.stack([-self.tangent[:, 1], self.tangent[:, 0]], axis=1)

        # sides: (s, 0) is side +, (s, 1) side -.  At vertex v, an incident segment leaves v in the
        # direction e; the side on the counter-clockwise hand of e is + if s starts at v, - if it ends
        # there.  Sector k lies between the k-th and (k+1)-th directions in counter-clockwise order.
        inc = defaultdict(list)
        for s in range(ns):
            inc[int(S[s, 0])].append((s, 0))
            inc[int(S[s, 1])].append((s, 1))
        self.q = np.zeros(nv, dtype=np.int64)
        self.side_sector = -np.ones((ns, 2, 2), dtype=np.int64)   # [s, end a, side]
        for v, lst in inc.items():
            items = []
            for s, a in lst:
                e = self.tangent[s] if a == 0 else -self.tangent[s]
                items.append((math.atan2(e[1], e[0]), s, a))
            items.sort()
            m = len(items)
            for k in range(m - 1):
                if items[k + 1][0] - items[k][0] < 1e-9:
                    raise MeshError2D("overlapping segments at a vertex")
            sectors = []
            for k in range(m):
                _, s1, a1 = items[k]
                _, s2, a2 = items[(k + 1) % m]
                ccw = (s1, 0 if a1 == 0 else 1)       # ccw hand of direction k
                cw = (s2, 1 if a2 == 0 else 0)        # cw hand of direction k+1
                sectors.append(sorted([ccw, cw]))
            order = sorted(range(m), key=lambda k: sectors[k][0])
            for label, k in enumerate(order):
                for (s, side) in sectors[k]:
                    a = 0 if int(S[s, 0]) == v else 1
                    self.side_sector[s, a, side] = label
            self.q[v] = m
        self.first_dof = np.zeros(nv + 1, dtype=np.int64)
        for v in range(nv):
            self.first_dof[v + 1] = self.first_dof[v] + max(int(self.q[v]) - 1, 0)
        self.N = int(self.first_dof[nv])
        self.dofs = [(v, j) for v in range(nv) for j in range(max(int(self.q[v]) - 1, 0))]
        # c[s, a, d]
        self.c = np.zeros((ns, 2, self.N))
        for s in range(ns):
            for a in range(2):
                v = int(S[s, a])
                qv = int(self.q[v])
                for j in range(qv - 1):
                    d = int(self.first_dof[v]) + j
                    sp = self.side_sector[s, a, 0]
                    sm = self.side_sector[s, a, 1]
                    tp = 1 if sp == j else (-1 if sp == qv - 1 else 0)
                    tm = 1 if sm == j else (-1 if sm == qv - 1 else 0)
                    self.c[s, a, d] = tp - tm

    def jump_values(self, phi):
        """jump[s, a]: the jump of sum_d phi_d psi_d across segment s at its end a."""
        return np.einsum("sad,d->sa", self.c, np.asarray(phi, dtype=np.float64))


def pair_integral(xa, xb, ya, yb, shared=None):
    """K = -1/(2 pi) int over [xa, xb] x [ya, yb] of log|x - y|.  shared: None (disjoint), 'same',
    or the common end as a pair (i, j) of indices 0/1 into (xa, xb) and (ya, yb)."""
    xa, xb, ya, yb = (np.asarray(p, dtype=np.float64) for p in (xa, xb, ya, yb))
    L1 = np.linalg.norm(xb - xa)
    L2 = np.linalg.norm(yb - ya)
    if shared == "same":
        return -(L1 * L1 * (math.log(L1) - 1.5)) / (2.0 * math.pi)
    if shared is None:
        t, w = gauss_legendre01(8)
        X = xa[None, :] + t[:, None] * (xb - xa)[None, :]
        Y = ya[None, :] + t[:, None] * (yb - ya)[None, :]
        r = np.linalg.norm(X[:, None, :] - Y[None, :, :], axis=2)
        return -(L1 * L2 * (w[:, None] * w[None, :] * np.log(r)).sum()) / (2.0 * math.pi)
    i, j = shared
    P = (xa, xb)[i]
    e1 = ((xb, xa)[i] - P) / L1
    e2 = ((yb, ya)[j] - P) / L2
    c = float(e1 @ e2)
    # int_0^1 int_0^1 log|L1 a e1 - L2 b e2| db da, split along a = b: each half is
    # int a log a da + (1/2) int a da int_0^1 log(...) d(eta) = -1/4 + (1/4) int_0^1 log(...) d(eta)
    A = _int_log_quadratic(L2 * L2, -2 * L1 * L2 * c, L1 * L1)
    B = _int_log_quadratic(L1 * L1, -2 * L1 * L2 * c, L2 * L2)
    return -(L1 * L2 * (-0.5 + 0.25 * (A + B))) / (2.0 * math.pi)


def _int_log_quadratic(a, b, c):
    """int_0^1 log(a x^2 + b x + c) dx for a quadratic without roots inside (0, 1): with
    a x^2 + b x + c = a ((x + p)^2 + q^2), the antiderivative of log(y^2 + q^2) is
    y log(y^2 + q^2) - 2 y + 2 q atan(y / q)."""
    p = b / (2.0 * a)
    q2 = max(c / a - p * p, 0.0)
    q = math.sqrt(q2)

    def F(y):
        v = y * y + q2
        out = (y * math.log(v) if v > 0 else 0.0) - 2.0 * y
        if q > 0:
            out += 2.0 * q * math.atan(y / q)
        return out

    return math.log(a) + F(1.0 + p) - F(p)


def pair_matrix(topo: Topology2D):
    V, S = topo.V, topo.S
    ns = topo.ns
    K = np.empty((ns, ns))
    for s in range(ns):
        for t in range(s, ns):
            if s == t:
                k = pair_integral(V[S[s, 0]], V[S[s, 1]], V[S[t, 0]], V[S[t, 1]], "same")
            else:
                common = [(i, j) for i in range(2) for j in range(2) if S[s, i] == S[t, j]]
                k = pair_integral(V[S[s, 0]], V[S[s, 1]], V[S[t, 0]], V[S[t, 1]], common[0] if common else None)
            K[s, t] = K[t, s] = k
    return K


def assemble(topo: Topology2D, K=None):
    """W = D^T K D with D[s, d] = (c[s,1,d] - c[s,0,d]) / |s|."""
    if K is None:
        K = pair_matrix(topo)
    D = (topo.c[:, 1, :] - topo.c[:, 0, :]) / topo.length[:, None]
    W = D.T @ K @ D
    return np.triu(W) + np.triu(W, 1).T      # each entry once, mirrored: exactly symmetric


def rhs(topo: Topology2D, g):
    """L[d, col] for constant fields g (k x 2 or 2)."""
    G = np.atleast_2d(np.asarray(g, dtype=np.float64))
    gn = G @ topo.normal.T                                   # k x ns
    csum = topo.c[:, 0, :] + topo.c[:, 1, :]                 # ns x N
    return -(csum.T @ (gn * (0.5 * topo.length)[None, :]).T)  # N x k


def double_layer(topo: Topology2D, jump, X):
    """U(x) = sum_s int_s n_s . (x - y) / (2 pi |x - y|^2) [u]_s(y) dy with 8-point Gauss-Legendre."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    J = np.asarray(jump, dtype=np.float64)
    t, w = gauss_legendre01(8)
    U = np.zeros(X.shape[0])
    for s in range(topo.ns):
        xa, xb = topo.V[topo.S[s, 0]], topo.V[topo.S[s, 1]]
        Y = xa[None, :] + t[:, None] * (xb - xa)[None, :]
        dens = (1 - t) * J[s, 0] + t * J[s, 1]
        d = X[:, None, :] - Y[None, :, :]
        r2 = (d * d).sum(axis=2)
        U += ((d @ topo.normal[s]) / (2 * math.pi * r2) * (w * dens * topo.length[s])[None, :]).sum(axis=1)
    return U


def cross_exact(X):
    """Experiment 1: U = Re(-1 / (2 i w)) with z = (w + 1/w)/2, |w| > 1."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    z = X[:, 0] + 1j * X[:, 1]
    w = z + np.sqrt(z - 1) * np.sqrt(z + 1)
    return np.real(-1.0 / (2j * w))


def classify_dofs_2d(topo: Topology2D, patch_of_segment):
    """Face dofs of patch P: dofs at vertices whose segments all lie in P and with q = 2; the rest
    form the wire basket (eq. jumpSplit in two dimensions)."""
    patch = np.asarray(patch_of_segment)
    seen = {}
    for s in range(topo.ns):
        for a in range(2):
            v = int(topo.S[s, a])
            p = int(patch[s]) if patch[s] >= 0 else -2
            seen[v] = p if seen.get(v, p) == p else -2
    faces = defaultdict(list)
    wb = []
    for d, (v, j) in enumerate(topo.dofs):
        if seen.get(v, -2) >= 0 and topo.q[v] == 2:
            faces[seen[v]].append(d)
        else:
            wb.append(d)
    return [faces[k] for k in sorted(faces)], wb


def coarse_prolongation_2d(fine: Topology2D, coarse: Topology2D, parent):
    """R_H (n_H x N): row (i, j) holds the fine coefficients of the coarse jump basis function
    psi^H_{i,j}.  On a coarse segment its traces are the coarse hat functions times the trace signs
    of psi^H_{i,j} at that end; at a fine vertex the per-sector values u_l give the coefficients
    u_l - mean(u) (the representative of the jump with sector values summing to zero)."""
    parent = np.asarray(parent)
    R = np.zeros((coarse.N, fine.N))
    # sector values of every coarse dof at every fine vertex
    vals = defaultdict(lambda: np.zeros(coarse.N))   # (fine vertex, fine sector) -> row over coarse dofs
    for s in range(fine.ns):
        S = int(parent[s])
        C0, C1 = coarse.V[coarse.S[S, 0]], coarse.V[coarse.S[S, 1]]
        same = float(fine.tangent[s] @ coarse.tangent[S]) > 0
        for a in range(2):
            v = int(fine.S[s, a])
            x = fine.V[v]
            l1 = float((x - C0) @ (C1 - C0)) / float((C1 - C0) @ (C1 - C0))
            lam = (1.0 - l1, l1)
            for side in range(2):
                key = (v, int(fine.side_sector[s, a, side]))
                if key in vals and vals[key].any():
                    continue
                cs = side if same else 1 - side
                row = np.zeros(coarse.N)
                for A in range(2):
                    if abs(lam[A]) < 1e-12:
                        continue
                    i = int(coarse.S[S, A])
                    qi = int(coarse.q[i])
                    jc = int(coarse.side_sector[S, A, cs])
                    for j in range(qi - 1):
                        sign = 1.0 if jc == j else (-1.0 if jc == qi - 1 else 0.0)
                        row[int(coarse.first_dof[i]) + j] += lam[A] * sign
                vals[key] = row
    for v in range(fine.nv):
        q = int(fine.q[v])
        if q < 2:
            continue
        U = np.stack([vals[(v, l)] if (v, l) in vals else np.zeros(coarse.N) for l in range(q)])   # q x nH
        coef = U - U.mean(axis=0)[None, :]
        for l in range(q - 1):
            R[:, int(fine.first_dof[v]) + l] = coef[l]
    return R
