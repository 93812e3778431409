"""Discrete jump space of a polygonal multiscreen mesh (test infrastructure; see oracle/__init__.py).

Follows Section 4.2 of the paper.  Around each mesh vertex x_i the region R^3 minus Gamma splits
into q_i connected sectors (the components of the star graph G(x_i), eqs. defCurlyHOmega /
defCurlyHGamma); each sector carries a split basis function phi_{i,j}.  The jump basis is
psi_{i,j} = phi_{i,j} - phi_{i,q_i} for j < q_i (eqs. defCurlyHtildeGamma, defYij), so there are
sum_i (q_i - 1) degrees of freedom.

The paper computes the sectors from the surface mesh alone by an "intrinsic inflation" algorithm
that it only cites.  Reading used here (no volume mesh): the sectors at x_i are the classes of the
sides (T, +/-) of the triangles T at x_i under the relation "bound the same wedge around an edge
at x_i".  Around an edge shared by several triangles the triangles are sorted by angle and the
side of each triangle facing the next one (cyclically) is joined with that next triangle's side
facing back; the two sides of a triangle at a free edge are joined.  Side "+" of T is the side
into which n_T = (x1-x0) x (x2-x0)/|.| points.

Labels: sectors at x_i are numbered by their smallest member, (triangle index, + before -), and
the last one is the reference sector q_i of eq. defYij.  Rejected inputs: degenerate or repeated
triangles, two triangles at an edge in the same half-plane (coincident pages) and point contacts
(the triangles at a vertex not connected through edges at that vertex; the paper excludes them,
footnote in Section 4.3).

Normal convention: the oriented triangle (T, side) carries the normal pointing out of the sector
on that side, i.e. n_(T,+) = -n_T and n_(T,-) = +n_T (the outward normal of the subdomain, as in
Thm. thmWweak and in the integration by parts behind l_g).
"""
from __future__ import annotations

import math
from collections import defaultdict

import numpy as np


class MeshError(ValueError):
    pass


def _find(parent, x):
    while parent[x] != x:
        parent[x] = parent[parent[x]]
        x = parent[x]
    return x


def _union(parent, a, b):
    ra, rb = _find(parent, a), _find(parent, b)
    if ra != rb:
        if ra < rb:
            parent[rb] = ra
        else:
            parent[ra] = rb


class Topology:
    """Sectors, degrees of freedom and jump coefficients of a triangle mesh."""

    def __init__(self, V, T, area_tol=1e-14):
        V = np.asarray(V, dtype=np.float64)
        T = np.asarray(T, dtype=np.int64)
        self.V, self.T = V, T
        nt, nv = T.shape[0], V.shape[0]
        self.nt, self.nv = nt, nv

        # ---- element geometry --------------------------------------------------------------
        e1 = V[T[:, 1]] - V[T[:, 0]]
        e2 = V[T[:, 2]] - V[T[:, 0]]
        cr = np.cross(e1, e2)
        twice_area = np.linalg.norm(cr, axis=1)
        scale = np.maximum(np.linalg.norm(e1, axis=1), np.linalg.norm(e2, axis=1)) ** 2
        if np.any(twice_area <= area_tol * scale):
            raise MeshError("degenerate triangle")
        self.area = 0.5 * twice_area
        self.normal = cr / twice_area[:, None]
        if len({tuple(sorted(t)) for t in T.tolist()}) != nt:
            raise MeshError("repeated triangle")

        # curl of the barycentric function lambda_a on T: n_T x grad lambda_a = (x_{a+1}-x_{a+2})/(2|T|)
        curl = np.empty((nt, 3, 3))
        for a in range(3):
            curl[:, a, :] = (V[T[:, (a + 1) % 3]] - V[T[:, (a + 2) % 3]]) / twice_area[:, None]
        self.curl = curl

        # ---- incidence ---------------------------------------------------------------------
        tris_at = defaultdict(list)
        for t in range(nt):
            for a in range(3):
                tris_at[int(T[t, a])].append(t)
        edges = defaultdict(list)
        for t in range(nt):
            for a in range(3):
                i, j = int(T[t, a]), int(T[t, (a + 1) % 3])
                edges[(min(i, j), max(i, j))].append(t)
        self.edges = edges

        # ---- per-edge wedge pairs ----------------------------------------------------------
        # side index: 2*t + s, s = 0 for '+', 1 for '-'
        joins = []   # (vertex-independent) pairs of sides that bound a common wedge at this edge
        for (i, j), tl in edges.items():
            if len(tl) == 1:
                t = tl[0]
                joins.append(((i, j), 2 * t, 2 * t + 1))
                continue
            xv, xw = V[i], V[j]
            e = xw - xv
            e = e / np.linalg.norm(e)
            items = []
            for t in tl:
                third = [int(k) for k in T[t] if k != i and k != j][0]
                d = V[third] - xv
                d = d - np.dot(d, e) * e
                items.append((t, d / np.linalg.norm(d)))
            b1 = items[0][1]
            b2 = np.cross(e, b1)
            ang = []
            for t, d in items:
                th = math.atan2(float(np.dot(d, b2)), float(np.dot(d, b1)))
                if th < 0:
                    th += 2.0 * math.pi
                ang.append((th, t, d))
            ang.sort()
            for k in range(len(ang)):
                th0, th1 = ang[k][0], ang[(k + 1) % len(ang)][0]
                gap = (th1 - th0) % (2.0 * math.pi)
                if gap < 1e-9 or gap > 2.0 * math.pi - 1e-9:
                    raise MeshError("coincident pages at an edge")
            for k in range(len(ang)):
                _, ta, da = ang[k]
                _, tb, db = ang[(k + 1) % len(ang)]
                # side of ta facing increasing angle: '+' iff n_ta . (e x d_ta) > 0
                inc_a = 0 if np.dot(self.normal[ta], np.cross(e, da)) > 0 else 1
                inc_b = 0 if np.dot(self.normal[tb], np.cross(e, db)) > 0 else 1
                dec_b = 1 - inc_b
                joins.append(((i, j), 2 * ta + inc_a, 2 * tb + dec_b))

        # ---- sectors at every vertex -------------------------------------------------------
        parent = {v: {} for v in tris_at}
        for v, tl in tris_at.items():
            for t in tl:
                parent[v][2 * t] = 2 * t
                parent[v][2 * t + 1] = 2 * t + 1
        for (i, j), sa, sb in joins:
            for v in (i, j):
                _union(parent[v], sa, sb)

        # point contacts: triangles at v must be connected through the edges at v
        for v, tl in tris_at.items():
            tp = {t: t for t in tl}
            for t in tl:
                for a in range(3):
                    i, j = int(T[t, a]), int(T[t, (a + 1) % 3])
                    if v in (i, j):
                        for t2 in edges[(min(i, j), max(i, j))]:
                            _union(tp, t, t2)
            if len({_find(tp, t) for t in tl}) > 1:
                raise MeshError("point contact at vertex %d" % v)

        self.q = np.zeros(nv, dtype=np.int64)
        # sector_of[(t, side, corner)] = label at vertex T[t, corner]
        self.sector = np.full((nt, 2, 3), -1, dtype=np.int64)
        for v, tl in tris_at.items():
            pv = parent[v]
            roots = {}
            for side in sorted(pv):           # members in (triangle, + before -) order
                r = _find(pv, side)
                if r not in roots:
                    roots[r] = len(roots)
            self.q[v] = len(roots)
            for t in tl:
                a = [k for k in range(3) if T[t, k] == v][0]
                for s in (0, 1):
                    self.sector[t, s, a] = roots[_find(pv, 2 * t + s)]

        # ---- degrees of freedom (vertex index, sector j < q-1), canonical order -------------
        dofs = []
        for v in range(nv):
            for j in range(int(self.q[v]) - 1):
                dofs.append((v, j))
        self.dofs = dofs
        self.N = len(dofs)
        self.dof_index = {d: k for k, d in enumerate(dofs)}

        # ---- jump coefficients c_{T,a,d} = s_(T,+) - s_(T,-) --------------------------------
        # trace of psi_{v,j} on side (T,s) at corner a: +1 if that side's sector is j, -1 if it
        # is the last sector q_v - 1, 0 otherwise
        self.tri_dofs = [[] for _ in range(nt)]     # per triangle: list of (dof, corner, c)
        for t in range(nt):
            for a in range(3):
                v = int(T[t, a])
                qv = int(self.q[v])
                for j in range(qv - 1):
                    s = []
                    for side in (0, 1):
                        sec = int(self.sector[t, side, a])
                        s.append(1 if sec == j else (-1 if sec == qv - 1 else 0))
                    c = s[0] - s[1]
                    if c != 0:
                        self.tri_dofs[t].append((self.dof_index[(v, j)], a, c))

    # ------------------------------------------------------------------------------------------
    def jump_vectors(self):
        """CSR over triangles: (ptr, dof, J) with J_{T,d} = sum_a c_{T,a,d} curl lambda_a^T."""
        ptr = [0]
        dof, J = [], []
        for t in range(self.nt):
            for (d, a, c) in self.tri_dofs[t]:
                dof.append(d)
                J.append(c * self.curl[t, a])
            ptr.append(len(dof))
        return (np.asarray(ptr, dtype=np.int64), np.asarray(dof, dtype=np.int64),
                np.asarray(J, dtype=np.float64).reshape(-1, 3))

    def jump_values(self, phi):
        """Label-free view of a coefficient vector: the jump of the represented function across T
        at each corner, jump[t, a] = sum_d c_{T,a,d} phi_d (trace on side + minus side -)."""
        out = np.zeros((self.nt, 3))
        for t in range(self.nt):
            for (d, a, c) in self.tri_dofs[t]:
                out[t, a] += c * phi[d]
        return out

    def q_histogram(self, nbins=16):
        h = np.zeros(nbins, dtype=np.int64)
        for qv in self.q:
            h[min(int(qv), nbins - 1)] += 1
        return h
