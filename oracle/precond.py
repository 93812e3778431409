"""Two-level substructuring additive Schwarz operator M (test infrastructure; see oracle/__init__.py).

Splitting of the discrete jump space (eq. jumpSplit, boxed in Section 6.4):
    V~_h = sum_F V~_F + V~_W + V~_H,
one copy per face (Remark after Def. proposedJumpSplit), and the action of M from the Remark
"Bound on the number of Preconditioned Conjugate Gradient iterations":
    M r = sum_X R_X^T (R_X W R_X^T)^{-1} R_X r,   X over faces, wire basket and coarse space.

Readings (the paper defines faces as coarse triangles; the workloads give patches):
  * face dofs of patch P: dofs at vertices all of whose triangles lie in P and with q = 2 (a
    patch-interior vertex of a flat region); every other dof is in the wire basket.  Both are
    spanned by fine jump basis functions, because the discrete harmonic extensions omega_{i,j}
    have the same traces as phi_{i,j} (Lemma lemdof and the line above it).
  * coarse space: the jump space of a nested coarse mesh, written in the fine basis.  A coarse
    split function phi^H_{i,j} takes, at a fine generalized vertex x_{k,l}, the value
    lambda^H_i(x_k) if the fine sector lies in coarse sector j of coarse vertex i, else 0; the
    fine coefficients of the jump of u are u_{k,l} - mean_l u_{k,.} for l < q_k (projection onto
    Psi_h along V_h(Omega), eq. orthogonalityVhYh).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .topology import Topology


def classify_dofs(topo: Topology, patch_of_triangle):
    """face_sets: list of arrays (one per patch with at least one face dof); wb: array."""
    patch_of_triangle = np.asarray(patch_of_triangle)
    T = topo.T
    vpatch = {}
    for t in range(topo.nt):
        p = int(patch_of_triangle[t])
        for a in range(3):
            v = int(T[t, a])
            if v not in vpatch:
                vpatch[v] = p
            elif vpatch[v] != p:
                vpatch[v] = -2          # touches two patches
    faces = {}
    wb = []
    for d, (v, j) in enumerate(topo.dofs):
        p = vpatch.get(v, -2)
        if p >= 0 and topo.q[v] == 2:
            faces.setdefault(p, []).append(d)
        else:
            wb.append(d)
    face_sets = [np.asarray(faces[p], dtype=np.int64) for p in sorted(faces)]
    return face_sets, np.asarray(wb, dtype=np.int64)


def coarse_prolongation(topo: Topology, coarse_V, coarse_T, coarse_of_triangle):
    """R_H (n_H x N): row (i,j) = fine coefficients of the coarse jump basis function psi^H_{i,j}."""
    ct = Topology(coarse_V, coarse_T)
    V, T = topo.V, topo.T
    cV, cT = ct.V, ct.T
    parent = np.asarray(coarse_of_triangle)
    R = np.zeros((ct.N, topo.N))
    # representative side of each fine sector: (vertex k, sector l) -> (triangle, side, corner)
    rep = {}
    for t in range(topo.nt):
        for a in range(3):
            k = int(T[t, a])
            for s in (0, 1):
                l = int(topo.sector[t, s, a])
                rep.setdefault((k, l), (t, s, a))
    for k in range(topo.nv):
        qk = int(topo.q[k])
        if qk < 2:
            continue
        u = {}    # coarse dof -> values over fine sectors l
        for l in range(qk):
            t, s, a = rep[(k, l)]
            tc = int(parent[t])
            sc = s if np.dot(topo.normal[t], ct.normal[tc]) > 0 else 1 - s
            # barycentric coordinates of x_k in the coarse triangle
            P0, P1, P2 = cV[cT[tc, 0]], cV[cT[tc, 1]], cV[cT[tc, 2]]
            M2 = np.stack([P1 - P0, P2 - P0], axis=1)
            lam12, *_ = np.linalg.lstsq(M2, V[k] - P0, rcond=None)
            lam = np.array([1.0 - lam12.sum(), lam12[0], lam12[1]])
            for ac in range(3):
                if abs(lam[ac]) < 1e-13:
                    continue
                i = int(cT[tc, ac])
                qi = int(ct.q[i])
                jc = int(ct.sector[tc, sc, ac])
                for j in range(qi - 1):
                    sign = 1.0 if jc == j else (-1.0 if jc == qi - 1 else 0.0)
                    if sign != 0.0:
                        u.setdefault(ct.dof_index[(i, j)], np.zeros(qk))[l] += lam[ac] * sign
        for cd, vals in u.items():
            cvals = vals - vals.mean()
            for l in range(qk - 1):
                if cvals[l] != 0.0:
                    R[cd, topo.dof_index[(k, l)]] = cvals[l]
    return R, ct


class AdditiveSchwarz:
    """M = sum_F R_F^T W_FF^{-1} R_F + R_W^T W_WW^{-1} R_W + R_H^T (R_H W R_H^T)^{-1} R_H.

    wirebasket="diagonal" replaces the Galerkin form on the wire-basket space by the pointwise
    (coefficient-wise) product weighted with the diagonal of W, so its subspace solver is
    R_W^T diag(W_WW)^{-1} R_W (Remark "Approximate solvers", Section 2: the bound of Thm. main
    survives a pointwise scalar product on the wire basket)."""

    def __init__(self, W, topo: Topology, patch_of_triangle=None, coarse_V=None, coarse_T=None,
                 coarse_of_triangle=None, face_sets=None, wb=None, use_coarse=True, wirebasket="exact", RH=None):
        if face_sets is None:
            face_sets, wb = classify_dofs(topo, patch_of_triangle)
        if wirebasket not in ("exact", "diagonal"):
            raise ValueError("wirebasket must be 'exact' or 'diagonal'")
        self.face_sets, self.wb = face_sets, wb
        self.blocks = []
        for idx in list(face_sets) + ([wb] if len(wb) and wirebasket == "exact" else []):
            self.blocks.append((idx, sla.cho_factor(W[np.ix_(idx, idx)], lower=True)))
        self.wb_diag = None
        if wirebasket == "diagonal" and len(wb):
            self.wb_diag = (np.asarray(wb), 1.0 / np.diag(W)[wb])
        self.RH = None
        if use_coarse and RH is not None:           # a coarse space given directly (segment meshes)
            self.RH = np.asarray(RH)
            self.WH = self.RH @ W @ self.RH.T
            self.WH_f = sla.cho_factor(self.WH, lower=True)
        elif use_coarse and coarse_V is not None:
            self.RH, self.coarse_topo = coarse_prolongation(topo, coarse_V, coarse_T, coarse_of_triangle)
            if self.RH.shape[0] > 0:
                self.WH = self.RH @ W @ self.RH.T
                self.WH_f = sla.cho_factor(self.WH, lower=True)
            else:
                self.RH = None

    def apply(self, r):
        z = np.zeros_like(r)
        for idx, f in self.blocks:
            z[idx] += sla.cho_solve(f, r[idx])
        if self.wb_diag is not None:
            idx, dinv = self.wb_diag
            z[idx] += dinv * r[idx]
        if self.RH is not None:
            z += self.RH.T @ sla.cho_solve(self.WH_f, self.RH @ r)
        return z

    def dense(self, N):
        return np.stack([self.apply(e) for e in np.eye(N)], axis=1)
