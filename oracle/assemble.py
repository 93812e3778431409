"""Galerkin matrix W and right-hand side L of the discrete problem W Phi = L (test infrastructure).

Section 4.3 of the paper: a(phi~_{i,j}, phi~_{i',j'}) is a double sum over oriented triangles of
curl . curl / (4 pi |x - x'|) (eq. eval_a_phiij with Cor. corW).  On an oriented triangle the trace
of psi_{v,j} is s * lambda_a with s in {+1, -1, 0}; its surface curl is s * n_(T,side) x grad
lambda_a, constant on T.  Summing the two sides of T with outward normals n_(T,+) = -n_T,
n_(T,-) = n_T gives -c_{T,a,d} curl lambda_a with c = s_+ - s_-, so

    W_{d,d'} = sum_{T,T'} I(T,T') J_{T,d} . J_{T',d'},   J_{T,d} = sum_a c_{T,a,d} curl lambda_a,

with I(T,T') = 1/(4 pi) int_T int_T' |x - y|^{-1} (the overall sign cancels in the product).
The right-hand side (eq. defRhs and the identity for l_g at the end of Section 4.3), constant g:

    L_d = sum_{(T,side)} int_T (g . n_(T,side)) s lambda_a = - sum_T (g . n_T) c_{T,a,d} |T| / 3.
"""
from __future__ import annotations

import numpy as np

from . import native
from .quadrature import gauss_legendre01, triangle7
from .topology import Topology

DEFAULT_NEAR_ORDER = 6


def _tables(near_order):
    bary, w = triangle7()
    gx, gw = gauss_legendre01(near_order)
    return (np.ascontiguousarray(bary, dtype=np.float64), np.ascontiguousarray(w, dtype=np.float64),
            np.ascontiguousarray(gx, dtype=np.float64), np.ascontiguousarray(gw, dtype=np.float64))


def pair_integrals(V, T, pairs, near_order=DEFAULT_NEAR_ORDER):
    """I(T,T') for the given (npairs, 2) index pairs (7x7 rule if disjoint, Duffy rules if touching)."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.int32)
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    b7, w7, gx, gw = _tables(near_order)
    out = np.empty(pairs.shape[0])
    native.lib().oracle_pair_integrals(native.dptr(V), native.iptr(T), native.dptr(b7), native.dptr(w7),
                                       near_order, native.dptr(gx), native.dptr(gw),
                                       pairs.shape[0], native.iptr(pairs), native.dptr(out))
    return out


def pair_matrix(V, T, near_order=DEFAULT_NEAR_ORDER):
    """The full N_T x N_T matrix of I(T,T') (small meshes only)."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.int32)
    nt = T.shape[0]
    b7, w7, gx, gw = _tables(near_order)
    out = np.empty((nt, nt))
    native.lib().oracle_I_rows(native.dptr(V), native.iptr(T), nt, native.dptr(b7), native.dptr(w7),
                               near_order, native.dptr(gx), native.dptr(gw), 0, nt, native.dptr(out))
    return out


def near_rule(kind, X, Y, near_order, kernel=0):
    """One Duffy-regularised rule on a touching pair.  kind: 'coincident' | 'edge' | 'vertex'.
    X, Y: (3,3) vertex arrays ordered so that shared vertices come first and match."""
    t = {"coincident": 3, "edge": 2, "vertex": 1}[kind]
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(9)
    Y = np.ascontiguousarray(Y, dtype=np.float64).reshape(9)
    gx, gw = gauss_legendre01(near_order)
    gx = np.ascontiguousarray(gx)
    gw = np.ascontiguousarray(gw)
    return native.lib().oracle_near_generic(t, native.dptr(X), native.dptr(Y), near_order,
                                            native.dptr(gx), native.dptr(gw), kernel)


def far_rule(X, Y, kernel=0):
    """7 x 7 product rule on a pair of triangles (any kernel id, see pairs.c)."""
    b7, w7, _, _ = _tables(2)
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(3, 3)
    Y = np.ascontiguousarray(Y, dtype=np.float64).reshape(3, 3)
    p = [np.ascontiguousarray(X[k]) for k in range(3)] + [np.ascontiguousarray(Y[k]) for k in range(3)]
    return native.lib().oracle_far_pair(*[native.dptr(a) for a in p], native.dptr(b7), native.dptr(w7), kernel)


class _JumpCSR:
    def __init__(self, topo: Topology):
        self.tri_ptr, self.tri_dof, self.tri_J = topo.jump_vectors()
        nt, N = topo.nt, topo.N
        # inverse CSR: dof -> (triangle, J)
        counts = np.bincount(self.tri_dof, minlength=N)
        self.dof_ptr = np.zeros(N + 1, dtype=np.int64)
        self.dof_ptr[1:] = np.cumsum(counts)
        self.dof_tri = np.empty(len(self.tri_dof), dtype=np.int64)
        self.dof_J = np.empty((len(self.tri_dof), 3))
        fill = self.dof_ptr[:-1].copy()
        tri_of_entry = np.repeat(np.arange(nt, dtype=np.int64), np.diff(self.tri_ptr))
        for e in range(len(self.tri_dof)):
            d = self.tri_dof[e]
            self.dof_tri[fill[d]] = tri_of_entry[e]
            self.dof_J[fill[d]] = self.tri_J[e]
            fill[d] += 1


def I_rows(V, T, r0, nrows, near_order=DEFAULT_NEAR_ORDER):
    """Rows r0 .. r0+nrows-1 of the N_T x N_T matrix of I(T,T') (all columns)."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.int32)
    nt = T.shape[0]
    b7, w7, gx, gw = _tables(near_order)
    out = np.empty((nrows, nt))
    native.lib().oracle_I_rows(native.dptr(V), native.iptr(T), nt, native.dptr(b7), native.dptr(w7),
                               near_order, native.dptr(gx), native.dptr(gw), r0, nrows, native.dptr(out))
    return out


def W_accumulate(topo: Topology, r0, I, d0, d1, csr=None):
    """The contraction step of `assemble` for one panel of rows of I (triangles r0 .. r0+len(I)-1):
    their contributions to rows d0 .. d1-1 of the upper triangle of W, as a (d1-d0) x N array."""
    c = csr or _JumpCSR(topo)
    I = np.ascontiguousarray(I, dtype=np.float64)
    out = np.zeros((d1 - d0, topo.N))
    native.lib().oracle_W_accumulate(topo.nt, topo.N, native.lptr(c.tri_ptr), native.lptr(c.tri_dof),
                                     native.dptr(np.ascontiguousarray(c.tri_J)), native.lptr(c.dof_ptr),
                                     native.lptr(c.dof_tri), native.dptr(c.dof_J), r0, I.shape[0],
                                     native.dptr(I), d0, d1, native.dptr(out))
    return out


def assemble(V, T, topo: Topology = None, near_order=DEFAULT_NEAR_ORDER, panel=1024):
    """Dense symmetric W (N x N) in canonical dof order."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.int32)
    topo = topo or Topology(V, T)
    c = _JumpCSR(topo)
    b7, w7, gx, gw = _tables(near_order)
    W = np.empty((topo.N, topo.N))
    native.lib().oracle_W(native.dptr(V), native.iptr(T), topo.nt, native.dptr(b7), native.dptr(w7),
                          near_order, native.dptr(gx), native.dptr(gw), topo.N,
                          native.lptr(c.tri_ptr), native.lptr(c.tri_dof), native.dptr(np.ascontiguousarray(c.tri_J)),
                          native.lptr(c.dof_ptr), native.lptr(c.dof_tri), native.dptr(c.dof_J),
                          panel, native.dptr(W))
    return W


def W_rows(V, T, rows, topo: Topology = None, near_order=DEFAULT_NEAR_ORDER):
    """Selected rows of W, each computed directly from the triangles of its dof's star."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.int32)
    topo = topo or Topology(V, T)
    c = _JumpCSR(topo)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    b7, w7, gx, gw = _tables(near_order)
    out = np.empty((rows.shape[0], topo.N))
    native.lib().oracle_W_rows(native.dptr(V), native.iptr(T), topo.nt, native.dptr(b7), native.dptr(w7),
                               near_order, native.dptr(gx), native.dptr(gw), topo.N,
                               native.lptr(c.tri_ptr), native.lptr(c.tri_dof), native.dptr(np.ascontiguousarray(c.tri_J)),
                               native.lptr(c.dof_ptr), native.lptr(c.dof_tri), native.dptr(c.dof_J),
                               rows.shape[0], native.lptr(rows), native.dptr(out))
    return out


def rhs(topo: Topology, g):
    """L (N x k) for k constant Neumann vectors g (k x 3):  L_d = -sum_T (g.n_T) c_{T,a,d} |T|/3."""
    g = np.atleast_2d(np.asarray(g, dtype=np.float64))
    L = np.zeros((topo.N, g.shape[0]))
    gn = topo.normal @ g.T            # (nt, k)
    for t in range(topo.nt):
        for (d, a, c) in topo.tri_dofs[t]:
            L[d] -= c * gn[t] * topo.area[t] / 3.0
    return L
