"""Seeded synthetic inputs: polygonal multiscreen meshes, patch partitions and nested coarse meshes.

This module only builds input arrays (vertex coordinates, triangle index triples, integer labels);
it holds none of the method's arithmetic.  Both the HIP path and the CPU oracle consume its output.

Geometries follow the workloads the paper describes in words (Section 2.2): flat screens, a
three-page "book" junction, three mutually perpendicular crossed panels (junction lines and a
junction point), the flat unit disk (a screen with a closed-form solution), the bow-tie of
Experiment 3, and random extruded multiscreens made of unit squares joined at shared edges.

Every panel is a parallelogram meshed by an ``nu x nv`` grid of cells, each cell split along its
(i,j)-(i+1,j+1) diagonal (or the other diagonal where a mirror-symmetric mesh is requested).  All
triangles of one panel share the normal ``u x v``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Panel:
    origin: Tuple[float, float, float]
    u: Tuple[float, float, float]
    v: Tuple[float, float, float]
    nu: int
    nv: int
    # cells whose diagonal runs (i+1,j)-(i,j+1) instead of (i,j)-(i+1,j+1): callable(i, j) -> bool
    anti_diag: Optional[object] = None


@dataclasses.dataclass
class Mesh:
    """A triangle mesh with per-triangle structure labels (panel, cell i, cell j, lower/upper)."""
    vertices: np.ndarray          # (nv, 3) float64
    triangles: np.ndarray         # (nt, 3) int32, vertex order fixes the normal
    tri_panel: np.ndarray         # (nt,) int32
    tri_cell: np.ndarray          # (nt, 2) int32 cell indices (i, j) inside the panel
    tri_lower: np.ndarray         # (nt,) bool: triangle on the u-side of the cell diagonal
    panels: List[Panel]

    @property
    def nv(self) -> int:
        return int(self.vertices.shape[0])

    @property
    def nt(self) -> int:
        return int(self.triangles.shape[0])


def _panel_point(p: Panel, i: int, j: int) -> Tuple[float, float, float]:
    a = i / p.nu
    b = j / p.nv
    return tuple(p.origin[k] + a * p.u[k] + b * p.v[k] for k in range(3))


def build_mesh(panels: Sequence[Panel], merge_tol: float = 1e-9) -> Mesh:
    """Mesh a list of panels and merge vertices that coincide (shared edges, junction lines)."""
    key_to_index = {}
    verts: List[Tuple[float, float, float]] = []
    tris: List[Tuple[int, int, int]] = []
    tri_panel: List[int] = []
    tri_cell: List[Tuple[int, int]] = []
    tri_lower: List[bool] = []
    scale = 1.0 / merge_tol

    def vid(pt):
        key = tuple(int(round(c * scale)) for c in pt)
        idx = key_to_index.get(key)
        if idx is None:
            idx = len(verts)
            key_to_index[key] = idx
            verts.append(pt)
        return idx

    for pid, p in enumerate(panels):
        grid = [[vid(_panel_point(p, i, j)) for j in range(p.nv + 1)] for i in range(p.nu + 1)]
        for i in range(p.nu):
            for j in range(p.nv):
                a, b, c, d = grid[i][j], grid[i + 1][j], grid[i + 1][j + 1], grid[i][j + 1]
                anti = bool(p.anti_diag(i, j)) if p.anti_diag is not None else False
                if not anti:
                    cell_tris = ((a, b, c, True), (a, c, d, False))
                else:
                    cell_tris = ((a, b, d, True), (b, c, d, False))
                for t0, t1, t2, low in cell_tris:
                    tris.append((t0, t1, t2))
                    tri_panel.append(pid)
                    tri_cell.append((i, j))
                    tri_lower.append(low)
    return Mesh(
        vertices=np.asarray(verts, dtype=np.float64).reshape(-1, 3),
        triangles=np.asarray(tris, dtype=np.int32).reshape(-1, 3),
        tri_panel=np.asarray(tri_panel, dtype=np.int32),
        tri_cell=np.asarray(tri_cell, dtype=np.int32).reshape(-1, 2),
        tri_lower=np.asarray(tri_lower, dtype=bool),
        panels=list(panels),
    )


# ----------------------------------------------------------------------------------------------
# Named geometries
# ----------------------------------------------------------------------------------------------

def unit_square(n: int) -> Mesh:
    """{0<=x,y<=1, z=0}, n x n cells (512 triangles and 225 interior vertices at n=16)."""
    return build_mesh([Panel((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), n, n)])


def rectangle(nx: int, ny: int, lx: float = 1.0, ly: float = 1.0) -> Mesh:
    return build_mesh([Panel((0.0, 0.0, 0.0), (lx, 0.0, 0.0), (0.0, ly, 0.0), nx, ny)])


def book(n: int, angles_deg: Sequence[float] = (0.0, 120.0, 240.0)) -> Mesh:
    """Unit-square pages sharing the spine {x=y=0, 0<=z<=1}; page k lies at azimuth angles_deg[k]."""
    panels = []
    for ang in angles_deg:
        th = math.radians(ang)
        u = (math.cos(th), math.sin(th), 0.0)
        # exact axis values for the common right angles keep mirror-symmetric inputs exact
        u = tuple(0.0 if abs(c) < 1e-15 else c for c in u)
        panels.append(Panel((0.0, 0.0, 0.0), u, (0.0, 0.0, 1.0), n, n))
    return build_mesh(panels)


def crossed(n: int, symmetric: bool = False) -> Mesh:
    """Squares [-1/2,1/2]^2 in the xy, yz and xz planes; n cells per unit length (n even).

    The coordinate axes are mesh lines of every panel they cross, so the three panels meet
    conformingly along the axes (junction lines, 4 sectors) and at the origin (8 sectors).
    With ``symmetric`` each quadrant's diagonals are mirrored so the mesh is invariant under the
    reflections of the coordinate planes.
    """
    if n % 2:
        raise ValueError("crossed(n) needs an even n so that the axes are mesh lines")
    h = n // 2

    def anti(i, j):
        return (i < h) != (j < h)

    a = anti if symmetric else None
    panels = [
        Panel((-0.5, -0.5, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), n, n, a),   # xy
        Panel((0.0, -0.5, -0.5), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0), n, n, a),   # yz
        Panel((-0.5, 0.0, -0.5), (1.0, 0.0, 0.0), (0.0, 0.0, 1.0), n, n, a),   # xz
    ]
    return build_mesh(panels)


def square_symmetric(n: int) -> Mesh:
    """[-1/2,1/2]^2 in the xy plane with per-quadrant mirrored diagonals (the xy panel of crossed)."""
    h = n // 2
    return build_mesh([Panel((-0.5, -0.5, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), n, n,
                             lambda i, j: (i < h) != (j < h))])


def bowtie(n: int) -> Mesh:
    """Two equal equilateral triangles in perpendicular planes sharing a common median.

    The median (length sqrt(3)/2) lies on the z axis from the apex (0,0,sqrt(3)/2) to the midpoint
    of the base (origin).  Each triangle is split by the median into two right triangles, each
    meshed as a half-grid; the pieces meet conformingly along the median.
    """
    hgt = math.sqrt(3.0) / 2.0
    verts = {}
    vlist: List[Tuple[float, float, float]] = []
    tris: List[Tuple[int, int, int]] = []
    pan: List[int] = []
    cell: List[Tuple[int, int]] = []
    low: List[bool] = []

    def vid(pt):
        key = tuple(int(round(c * 1e9)) for c in pt)
        if key not in verts:
            verts[key] = len(vlist)
            vlist.append(pt)
        return verts[key]

    # each half: right triangle with legs along the base direction d (length 1/2) and z (length hgt)
    halves = [(1.0, 0.0, 0.0), (-1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, -1.0, 0.0)]
    for pid, d in enumerate(halves):
        def pt(i, j):
            # i along the base (0..n), j up the median (0..n); only i + j <= n is inside
            x = 0.5 * (i / n)
            z = hgt * (j / n)
            return (d[0] * x, d[1] * x, z)
        for i in range(n):
            for j in range(n - i):
                a, b, c = vid(pt(i, j)), vid(pt(i + 1, j)), vid(pt(i, j + 1))
                tris.append((a, b, c)); pan.append(pid); cell.append((i, j)); low.append(True)
                if i + j + 1 < n:
                    d2 = vid(pt(i + 1, j + 1))
                    tris.append((b, d2, c)); pan.append(pid); cell.append((i, j)); low.append(False)
    return Mesh(np.asarray(vlist, dtype=np.float64), np.asarray(tris, dtype=np.int32),
                np.asarray(pan, dtype=np.int32), np.asarray(cell, dtype=np.int32).reshape(-1, 2),
                np.asarray(low, dtype=bool), [])


def bowtie_coarse(n: int, ratio: int) -> Tuple[Mesh, np.ndarray]:
    """Nested coarse mesh of bowtie(n): bowtie(n // ratio), and the coarse triangle of each fine one.

    Cells are split on their (i+1, j)-(i, j+1) diagonal at both levels, so a fine triangle of cell
    (i, j) lies in coarse cell (i // ratio, j // ratio), below the coarse diagonal when its offsets
    (a, b) in that cell have a + b < ratio - 1, or a + b = ratio - 1 and it is the lower fine one.
    """
    if n % ratio:
        raise ValueError("ratio must divide n")
    fine, cm = bowtie(n), bowtie(n // ratio)
    lookup = {}
    for t in range(cm.nt):
        lookup[(int(cm.tri_panel[t]), int(cm.tri_cell[t, 0]), int(cm.tri_cell[t, 1]), bool(cm.tri_lower[t]))] = t
    parent = np.empty(fine.nt, dtype=np.int32)
    for t in range(fine.nt):
        i, j = int(fine.tri_cell[t, 0]), int(fine.tri_cell[t, 1])
        I, J = i // ratio, j // ratio
        s = (i - I * ratio) + (j - J * ratio)
        lower = s < ratio - 1 or (s == ratio - 1 and bool(fine.tri_lower[t]))
        parent[t] = lookup[(int(fine.tri_panel[t]), I, J, lower)]
    return cm, parent


# Neumann data of the paper's three-dimensional experiment (two perpendicular triangles)
BOWTIE_G = np.array([1.0, 0.5, 0.25])


def fan(m: int, rings: int = 2) -> Mesh:
    """Unit disk in the plane z=0 meshed by m spokes: every ring k = 1..rings holds m vertices, so the
    centre vertex sits in m thin triangles (a star far longer than a structured mesh's)."""
    vlist: List[Tuple[float, float, float]] = [(0.0, 0.0, 0.0)]
    for k in range(1, rings + 1):
        r = k / rings
        for i in range(m):
            th = 2.0 * math.pi * i / m
            vlist.append((r * math.cos(th), r * math.sin(th), 0.0))

    def ring(k, i):
        return 0 if k == 0 else 1 + (k - 1) * m + (i % m)

    tris: List[Tuple[int, int, int]] = []
    for i in range(m):
        tris.append((0, ring(1, i), ring(1, i + 1)))
    for k in range(1, rings):
        for i in range(m):
            a0, a1, b0, b1 = ring(k, i), ring(k, i + 1), ring(k + 1, i), ring(k + 1, i + 1)
            tris.append((a0, b0, b1))
            tris.append((a0, b1, a1))
    V = np.asarray(vlist, dtype=np.float64)
    T = np.asarray(tris, dtype=np.int32)
    nt = T.shape[0]
    return Mesh(V, T, np.zeros(nt, np.int32), np.zeros((nt, 2), np.int32), np.zeros(nt, bool), [])


def disk(m: int) -> Mesh:
    """Unit disk in the plane z=0: m concentric rings, ring k holding 6k vertices (normal +z)."""
    vlist: List[Tuple[float, float, float]] = [(0.0, 0.0, 0.0)]
    rings = [[0]]
    for k in range(1, m + 1):
        r = k / m
        ring = []
        for i in range(6 * k):
            th = 2.0 * math.pi * i / (6 * k)
            ring.append(len(vlist))
            vlist.append((r * math.cos(th), r * math.sin(th), 0.0))
        rings.append(ring)
    tris: List[Tuple[int, int, int]] = []
    for k in range(1, m + 1):
        inner, outer = rings[k - 1], rings[k]
        ni, no = len(inner), len(outer)
        if ni == 1:
            for i in range(no):
                tris.append((inner[0], outer[i], outer[(i + 1) % no]))
            continue
        # two-pointer sweep by angle around the annulus
        ia, ib = 0, 0
        while ia < ni or ib < no:
            a_next = (ia + 1) / ni
            b_next = (ib + 1) / no
            if ib < no and (ia >= ni or b_next <= a_next):
                tris.append((inner[ia % ni], outer[ib % no], outer[(ib + 1) % no]))
                ib += 1
            else:
                tris.append((inner[ia % ni], outer[ib % no], inner[(ia + 1) % ni]))
                ia += 1
    V = np.asarray(vlist, dtype=np.float64)
    T = np.asarray(tris, dtype=np.int32)
    # orient every triangle with normal +z
    e1 = V[T[:, 1]] - V[T[:, 0]]
    e2 = V[T[:, 2]] - V[T[:, 0]]
    flip = (e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    nt = T.shape[0]
    return Mesh(V, T, np.zeros(nt, np.int32), np.zeros((nt, 2), np.int32), np.zeros(nt, bool), [])


# ----------------------------------------------------------------------------------------------
# Extruded random multiscreens (serving stream): unit segments in the xy plane, extruded in z
# ----------------------------------------------------------------------------------------------

def _segments_intersect(p1, p2, q1, q2, eps=1e-9):
    def orient(a, b, c):
        return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])

    def on_seg(a, b, c):
        return (min(a[0], b[0]) - eps <= c[0] <= max(a[0], b[0]) + eps and
                min(a[1], b[1]) - eps <= c[1] <= max(a[1], b[1]) + eps)

    d1, d2 = orient(q1, q2, p1), orient(q1, q2, p2)
    d3, d4 = orient(p1, p2, q1), orient(p1, p2, q2)
    if ((d1 > eps and d2 < -eps) or (d1 < -eps and d2 > eps)) and \
       ((d3 > eps and d4 < -eps) or (d3 < -eps and d4 > eps)):
        return True
    if abs(d1) <= eps and on_seg(q1, q2, p1):
        return True
    if abs(d2) <= eps and on_seg(q1, q2, p2):
        return True
    if abs(d3) <= eps and on_seg(p1, p2, q1):
        return True
    if abs(d4) <= eps and on_seg(p1, p2, q2):
        return True
    return False


def _pt_seg_dist(p, a, b):
    ax, ay = b[0] - a[0], b[1] - a[1]
    t = ((p[0] - a[0]) * ax + (p[1] - a[1]) * ay) / (ax * ax + ay * ay)
    t = min(1.0, max(0.0, t))
    dx, dy = a[0] + t * ax - p[0], a[1] + t * ay - p[1]
    return math.hypot(dx, dy)


def random_extruded(rng: np.random.Generator, n_squares: int, layout: str, n: int,
                    max_tries: int = 200) -> Tuple[Mesh, dict]:
    """1-6 unit squares joined at shared vertical edges, dihedral angles uniform in [30, 330] deg.

    The cross-section in the xy plane is a graph of unit segments (book: all share one node;
    chain: a polyline; tree: each new segment hangs off a random existing node).  Layouts whose
    segments cross, overlap or touch away from shared nodes are rejected and redrawn.
    """
    for _ in range(max_tries):
        nodes = [(0.0, 0.0)]
        segs: List[Tuple[int, int]] = []
        heading = {0: 0.0}
        ok = True
        for s in range(n_squares):
            if layout == "book" or s == 0:
                base = 0
            elif layout == "chain":
                base = len(nodes) - 1
            else:
                base = int(rng.integers(0, len(nodes)))
            dih = math.radians(float(rng.uniform(30.0, 330.0)))
            ang = heading.get(base, 0.0) + (math.pi - dih if s > 0 else 0.0)
            if layout == "book" and s > 0:
                ang = float(rng.uniform(0.0, 2.0 * math.pi))
            p0 = nodes[base]
            p1 = (p0[0] + math.cos(ang), p0[1] + math.sin(ang))
            # reject: new segment meets an old one anywhere but at the shared node, or lies closer
            # than 30 degrees (about 0.5 units) to another segment end
            for (a, b) in segs:
                pa, pb = nodes[a], nodes[b]
                shared = base in (a, b)
                if shared:
                    other = pb if a == base else pa
                    d0 = (other[0] - p0[0], other[1] - p0[1])
                    d1 = (p1[0] - p0[0], p1[1] - p0[1])
                    cosang = (d0[0] * d1[0] + d0[1] * d1[1])
                    if cosang > math.cos(math.radians(29.9)):
                        ok = False
                        break
                    if _pt_seg_dist(p1, pa, pb) < 0.2:
                        ok = False
                        break
                else:
                    if _segments_intersect(p0, p1, pa, pb) or min(
                            _pt_seg_dist(p0, pa, pb), _pt_seg_dist(p1, pa, pb),
                            _pt_seg_dist(pa, p0, p1), _pt_seg_dist(pb, p0, p1)) < 0.2:
                        ok = False
                        break
            if not ok:
                break
            nodes.append(p1)
            heading[len(nodes) - 1] = ang
            segs.append((base, len(nodes) - 1))
        if not ok:
            continue
        panels = []
        for (a, b) in segs:
            pa, pb = nodes[a], nodes[b]
            panels.append(Panel((pa[0], pa[1], 0.0), (pb[0] - pa[0], pb[1] - pa[1], 0.0),
                                (0.0, 0.0, 1.0), n, n))
        return build_mesh(panels), {"nodes": nodes, "segments": segs, "layout": layout}
    raise RuntimeError("could not draw a valid extruded multiscreen")


# ----------------------------------------------------------------------------------------------
# Patch partitions and nested coarse meshes (inputs of the preconditioner set-up)
# ----------------------------------------------------------------------------------------------

def grid_patches(mesh: Mesh, cells_per_patch: int, split_at: Optional[Sequence[int]] = None) -> np.ndarray:
    """Square patches of cells_per_patch x cells_per_patch cells on every panel.

    ``split_at``: extra cut lines (cell indices) applied on both panel axes, so patches never
    straddle junction lines that cross a panel (the coordinate axes of the crossed geometry).
    """
    out = np.empty(mesh.nt, dtype=np.int32)
    next_id = 0
    for pid, p in enumerate(mesh.panels):
        def cuts(nc):
            c = set(range(0, nc + 1, cells_per_patch)) | {nc}
            if split_at is not None:
                c |= set(s for s in split_at if 0 < s < nc)
            return sorted(c)
        cu, cv = cuts(p.nu), cuts(p.nv)
        sel = np.nonzero(mesh.tri_panel == pid)[0]
        iu = np.searchsorted(cu, mesh.tri_cell[sel, 0], side="right") - 1
        iv = np.searchsorted(cv, mesh.tri_cell[sel, 1], side="right") - 1
        out[sel] = next_id + iu * (len(cv) - 1) + iv
        next_id += (len(cu) - 1) * (len(cv) - 1)
    return out


def guillotine_patches(mesh: Mesh, rng: np.random.Generator, blocks_per_panel_axis: int,
                       patches_per_block: int, dof_range: Tuple[int, int],
                       max_tries: int = 1000) -> np.ndarray:
    """Seeded random guillotine partition (uneven patch sizes).

    Each panel is first cut into blocks_per_panel_axis^2 equal blocks (for the crossed geometry
    these are the quadrants cut out by the junction lines); each block is split recursively, at a
    fraction uniform in [0.3, 0.7] along its longer side, into patches_per_block rectangles.  A
    block's split is redrawn until every rectangle's interior vertex count lies in dof_range.
    """
    out = np.empty(mesh.nt, dtype=np.int32)
    next_id = 0
    for pid, p in enumerate(mesh.panels):
        bu, bv = p.nu // blocks_per_panel_axis, p.nv // blocks_per_panel_axis
        sel = np.nonzero(mesh.tri_panel == pid)[0]
        ci, cj = mesh.tri_cell[sel, 0], mesh.tri_cell[sel, 1]
        for bi in range(blocks_per_panel_axis):
            for bj in range(blocks_per_panel_axis):
                for _ in range(max_tries):
                    rects = [(bi * bu, bj * bv, bu, bv)]
                    while len(rects) < patches_per_block:
                        rects.sort(key=lambda r: -r[2] * r[3])
                        x, y, w, h = rects.pop(0)
                        f = float(rng.uniform(0.3, 0.7))
                        if w >= h:
                            k = max(1, min(w - 1, int(round(f * w))))
                            rects += [(x, y, k, h), (x + k, y, w - k, h)]
                        else:
                            k = max(1, min(h - 1, int(round(f * h))))
                            rects += [(x, y, w, k), (x, y + k, w, h - k)]
                    if all(dof_range[0] <= (w - 1) * (h - 1) <= dof_range[1] for (_, _, w, h) in rects):
                        break
                else:
                    raise RuntimeError("guillotine partition: no admissible split found")
                for (x, y, w, h) in rects:
                    m = (ci >= x) & (ci < x + w) & (cj >= y) & (cj < y + h)
                    out[sel[m]] = next_id
                    next_id += 1
    return out


def coarse_mesh(mesh: Mesh, ratio: int) -> Tuple[Mesh, np.ndarray]:
    """Nested coarse mesh: every panel re-meshed with cells ratio times larger, same diagonals.

    Returns the coarse mesh and coarse_of_triangle (the coarse triangle containing each fine one).
    The fine mesh must have been built from the same panels with nu, nv divisible by ratio and a
    diagonal pattern that is constant on each coarse cell.
    """
    cpanels = []
    for p in mesh.panels:
        if p.nu % ratio or p.nv % ratio:
            raise ValueError("coarse ratio must divide the panel cell counts")
        ad = None
        if p.anti_diag is not None:
            f = p.anti_diag
            ad = (lambda f_: (lambda I, J: f_(I * ratio, J * ratio)))(f)
        cpanels.append(Panel(p.origin, p.u, p.v, p.nu // ratio, p.nv // ratio, ad))
    cm = build_mesh(cpanels)
    # index of coarse triangles: (panel, I, J, lower) -> id
    lookup = {}
    for t in range(cm.nt):
        lookup[(int(cm.tri_panel[t]), int(cm.tri_cell[t, 0]), int(cm.tri_cell[t, 1]),
                bool(cm.tri_lower[t]))] = t
    parent = np.empty(mesh.nt, dtype=np.int32)
    for t in range(mesh.nt):
        pid = int(mesh.tri_panel[t])
        i, j = int(mesh.tri_cell[t, 0]), int(mesh.tri_cell[t, 1])
        I, J = i // ratio, j // ratio
        a, b = i - I * ratio, j - J * ratio
        anti = False
        p = mesh.panels[pid]
        if p.anti_diag is not None:
            anti = bool(p.anti_diag(i, j))
        if not anti:
            # coarse diagonal (0,0)-(r,r): lower side is a > b
            lower = (a > b) or (a == b and bool(mesh.tri_lower[t]))
        else:
            # coarse diagonal (r,0)-(0,r): lower side is a + b < r - 1, or on it the fine lower one
            s = a + b
            lower = (s < ratio - 1) or (s == ratio - 1 and bool(mesh.tri_lower[t]))
        parent[t] = lookup[(pid, I, J, lower)]
    return cm, parent


def unit_g(seed: int) -> np.ndarray:
    """Neumann data: a unit vector drawn from numpy.random.default_rng(seed)."""
    g = np.random.default_rng(seed).standard_normal(3)
    return g / np.linalg.norm(g)


# ----------------------------------------------------------------------------------------------
# Workload presets
# ----------------------------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    mesh: Mesh
    patch_of_triangle: np.ndarray
    coarse: Mesh
    coarse_of_triangle: np.ndarray
    g: np.ndarray                 # (k, 3)
    description: str


def workload(name: str, seed: int = 0, k: int = 1) -> Workload:
    """The named synthetic workloads.

    square16   unit square, 16x16 cells, g=(0,0,1), 2x2 square patches, coarse H=1/2
    book48     three-page book at 0/120/240 deg, h=1/48, 4x4 patches per page, coarse H=1/4
    crossed96  crossed panels, h=1/96, 96 random guillotine patches (150-500 dofs), coarse H=1/8
    crossed192 crossed panels, h=1/192, 384 random patches (about 16x16 cells), coarse H=1/12
    """
    rng = np.random.default_rng(seed)
    if name == "square16":
        m = unit_square(16)
        patches = grid_patches(m, 8)
        cm, par = coarse_mesh(m, 8)
        g = np.tile(np.array([0.0, 0.0, 1.0]), (k, 1))
        desc = "unit square, 16x16 cells, 2x2 patches (H/h=8), coarse H=1/2"
    elif name == "book48":
        m = book(48)
        patches = grid_patches(m, 12)
        cm, par = coarse_mesh(m, 12)
        g = np.stack([unit_g(seed + i) for i in range(k)])
        desc = "three-page book 0/120/240 deg, h=1/48, 48 square patches (H/h=12), coarse H=1/4"
    elif name == "crossed96":
        m = crossed(96)
        patches = guillotine_patches(m, rng, 2, 8, (150, 500))
        cm, par = coarse_mesh(m, 12)
        g = np.stack([unit_g(seed + i) for i in range(k)])
        desc = "crossed panels, h=1/96, 96 random guillotine patches (150-500 dofs), coarse H=1/8"
    elif name == "crossed192":
        m = crossed(192)
        patches = guillotine_patches(m, rng, 2, 32, (100, 400))
        cm, par = coarse_mesh(m, 16)
        g = np.stack([unit_g(seed + i) for i in range(k)])
        desc = "crossed panels, h=1/192, 384 random patches (H/h~16), coarse H=1/12"
    else:
        raise KeyError(name)
    return Workload(name, m, patches, cm, par, g, desc)


# ----------------------------------------------------------------------------------------------
# Serving stream: seeded Poisson arrivals of solve requests on random multiscreens
# ----------------------------------------------------------------------------------------------

@dataclasses.dataclass
class ServeRequest:
    t_arrival: float              # seconds after the start of the stream
    geometry: int                 # index of the geometry (requests on one geometry share it)
    mesh: Mesh
    patch_of_triangle: np.ndarray
    coarse: Mesh
    coarse_of_triangle: np.ndarray
    g: np.ndarray                 # (k, 3) unit vectors
    mixed: bool                   # FP32 matrix + FP64 refinement, else plain FP64


def serving_stream(seed: int, n_requests: int, rate: float, n_range: Tuple[int, int] = (2000, 30000),
                   k_range: Tuple[int, int] = (1, 16), cells_per_patch: int = 15,
                   reuse: float = 0.5) -> List[ServeRequest]:
    """Requests arriving as a Poisson process of the given rate (per second).

    Each new geometry is 1-6 unit squares joined at shared edges (book, chain or tree layout,
    dihedral angles uniform in [30, 330] deg) with m x m square patches of cells_per_patch cells
    per panel, m chosen so that the dof count is near a target drawn uniformly from n_range, and a
    nested coarse mesh with one coarse cell per patch; it is served in FP64 or in mixed precision
    with equal probability (fixed per geometry: a resident problem keeps its precision).  With
    probability ``reuse`` a request reuses one of the three most recent geometries (new right-hand
    sides on a resident problem, arriving in bursts).  Each request has k ~ U{k_range} random unit g.
    """
    rng = np.random.default_rng(seed)
    geos: List[Tuple[Mesh, np.ndarray, Mesh, np.ndarray, bool]] = []
    out: List[ServeRequest] = []
    t = 0.0
    c = cells_per_patch
    for _ in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        if geos and rng.uniform() < reuse:
            gi = len(geos) - 1 - int(rng.integers(0, min(3, len(geos))))
        else:
            n_sq = int(rng.integers(1, 7))
            layout = str(rng.choice(["book", "chain", "tree"]))
            target = float(rng.uniform(*n_range))
            m_side = max(2, int(round(math.sqrt(target / n_sq) / c)))
            mesh, _ = random_extruded(rng, n_sq, layout, c * m_side)
            cm, par = coarse_mesh(mesh, c)
            geos.append((mesh, grid_patches(mesh, c), cm, par, bool(rng.integers(0, 2))))
            gi = len(geos) - 1
        mesh, patches, cm, par, mixed = geos[gi]
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        g = rng.standard_normal((k, 3))
        g /= np.linalg.norm(g, axis=1, keepdims=True)
        out.append(ServeRequest(t, gi, mesh, patches, cm, par, g, mixed))
    return out


# ---- two-dimensional multiscreens (segment meshes in the plane) ----------------------------------

def _arms_mesh(center, tips, n, grading=1.0):
    """Segments from a common centre to each tip, n per arm; grading > 1 refines towards the tips
    (node k at 1 - (1 - k/n)^grading of the arm)."""
    V = [tuple(center)]
    S = []
    for tip in tips:
        prev = 0
        for k in range(1, n + 1):
            s = 1.0 - (1.0 - k / n) ** grading
            V.append(tuple(np.asarray(center) + s * (np.asarray(tip) - np.asarray(center))))
            S.append((prev, len(V) - 1))
            prev = len(V) - 1
    return np.asarray(V, dtype=np.float64), np.asarray(S, dtype=np.int32)


def plus2d(n: int, grading: float = 1.0):
    """Experiment 1: the cross [-1, 1] x {0} u {0} x [-1, 1], n segments per arm."""
    return _arms_mesh((0.0, 0.0), [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)], n, grading)


def threefold2d(n: int):
    """Experiment 2: three segments from the centre of gravity of an equilateral triangle (side 1)
    to its vertices, n segments each."""
    r = 1.0 / math.sqrt(3.0)
    tips = [(r * math.cos(a), r * math.sin(a)) for a in (math.pi / 2, math.pi / 2 + 2 * math.pi / 3,
                                                         math.pi / 2 + 4 * math.pi / 3)]
    return _arms_mesh((0.0, 0.0), tips, n)


def slit2d(n: int):
    """The segment [-1, 1] x {0} with 2n segments (nodes at the cross's horizontal-arm nodes)."""
    x = np.linspace(-1.0, 1.0, 2 * n + 1)
    V = np.stack([x, np.zeros_like(x)], axis=1)
    S = np.stack([np.arange(2 * n), np.arange(1, 2 * n + 1)], axis=1).astype(np.int32)
    return V, S


def arms2d_coarse(kind: str, n: int, ratio: int):
    """Nested coarse mesh of plus2d(n) / threefold2d(n): the same arms with n // ratio segments,
    and coarse_of_segment (fine segment k of an arm lies in coarse segment k // ratio)."""
    if n % ratio:
        raise ValueError("ratio must divide n")
    gen = {"plus": plus2d, "threefold": threefold2d}[kind]
    V, S = gen(n)
    cV, cS = gen(n // ratio)
    arms = S.shape[0] // n
    parent = np.array([a * (n // ratio) + k // ratio for a in range(arms) for k in range(n)], dtype=np.int32)
    return (V, S), (cV, cS), parent


def cross_solution(X):
    """Experiment 1's reference field on the plus-shaped cross: U = Re(-1 / (2 i w)) with
    z = x1 + i x2 = (w + 1/w) / 2, |w| > 1 (the potential of the dipole density sqrt(1 - x1^2) on the
    horizontal arm; its Neumann data on the cross are those of the constant field g = (0, -1/2))."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    z = X[:, 0] + 1j * X[:, 1]
    w = z + np.sqrt(z - 1.0) * np.sqrt(z + 1.0)
    return np.real(-1.0 / (2j * w))
