"""Pins of the oracle's sectors / dofs / jump coefficients (CPU only).

Counting facts: a flat interior vertex has q = 2 sectors, a screen-boundary vertex q = 1, a vertex
on the spine of a three-page book q = 3, on a line where two planes cross q = 4, at the point
where three planes cross q = 8; the number of dofs is sum_i (q_i - 1) (Section 4.2).
"""
import math

import numpy as np
import pytest

from paper_2310_09204_amd import meshes
from oracle.topology import MeshError, Topology


def q_at(topo, point):
    d = np.linalg.norm(topo.V - np.asarray(point), axis=1)
    return int(topo.q[int(np.argmin(d))])


def test_flat_square_counts():
    m = meshes.unit_square(16)
    t = Topology(m.vertices, m.triangles)
    assert t.N == 225
    assert q_at(t, (0.5, 0.5, 0)) == 2 and q_at(t, (0.0, 0.5, 0)) == 1 and q_at(t, (1, 1, 0)) == 1
    assert sum(int(q) - 1 for q in t.q if q > 0) == t.N


def test_book_counts():
    m = meshes.book(8)
    t = Topology(m.vertices, m.triangles)
    assert q_at(t, (0, 0, 0.5)) == 3
    assert q_at(t, (0, 0, 0.0)) == 1          # spine end on the boundary
    # 3 pages of 7x7 interior vertices plus 7 spine vertices with 2 dofs each
    assert t.N == 3 * 7 * 7 + 7 * 2


def test_book48_count():
    m = meshes.book(48)
    t = Topology(m.vertices, m.triangles)
    assert t.N == 3 * 47 * 47 + 47 * 2 == 6721


@pytest.mark.parametrize("n", [4, 8, 12])
def test_crossed_counts(n):
    m = meshes.crossed(n)
    t = Topology(m.vertices, m.triangles)
    assert q_at(t, (0, 0, 0)) == 8
    assert q_at(t, (0.25, 0, 0)) == 4 and q_at(t, (0, 0.25, 0)) == 4 and q_at(t, (0, 0, -0.25)) == 4
    assert q_at(t, (0.5, 0, 0)) == 1
    expected = 3 * ((n - 1) ** 2 - (2 * n - 3)) + 9 * (n - 2) + 7
    assert t.N == expected


def test_fin_on_a_square():
    # a vertical fin standing on the middle line of a flat square: three sheets meet along the
    # line (q = 3), the fin's free top edge has q = 1
    panels = [meshes.Panel((0, 0, 0), (0.5, 0, 0), (0, 1, 0), 4, 8),
              meshes.Panel((0.5, 0, 0), (0.5, 0, 0), (0, 1, 0), 4, 8),
              meshes.Panel((0.5, 0, 0), (0, 0, 0.5), (0, 1, 0), 4, 8)]
    m = meshes.build_mesh(panels)
    t = Topology(m.vertices, m.triangles)
    assert q_at(t, (0.5, 0.5, 0)) == 3
    assert q_at(t, (0.5, 0.5, 0.5)) == 1
    assert q_at(t, (0.5, 0.5, 0.25)) == 2


def test_flat_screen_jump_coefficients_are_two():
    m = meshes.unit_square(6)
    t = Topology(m.vertices, m.triangles)
    for lst in t.tri_dofs:
        for (_, _, c) in lst:
            assert c == 2


def test_rejections():
    V = np.array([[0., 0, 0], [1, 0, 0], [0, 1, 0], [2, 0, 0], [0, 0, 1]])
    with pytest.raises(MeshError):
        Topology(V, np.array([[0, 1, 3]]))                     # degenerate (collinear)
    with pytest.raises(MeshError):
        Topology(V, np.array([[0, 1, 2], [1, 2, 0]]))          # repeated triangle
    # two pages of a book in the same half-plane
    V2 = np.array([[0., 0, 0], [0, 0, 1], [1, 0, 0], [2, 0, 0.5]])
    with pytest.raises(MeshError):
        Topology(V2, np.array([[0, 1, 2], [0, 1, 3]]))
    # point contact: two triangles touching at one vertex only
    V3 = np.array([[0., 0, 0], [1, 0, 0], [0, 1, 0], [-1, 0, 0.3], [0, -1, 0.2]])
    with pytest.raises(MeshError):
        Topology(V3, np.array([[0, 1, 2], [0, 3, 4]]))


def test_jump_values_label_free_on_book_rotation():
    # the page permutation of a rotationally symmetric book maps sectors to sectors
    m = meshes.book(4)
    t = Topology(m.vertices, m.triangles)
    assert t.N == 3 * 9 + 3 * 2
    assert int(t.q_histogram()[3]) == 3
