"""The library's host-side sector analysis (C++) agrees exactly with the oracle's (numpy), and
rejects invalid meshes with the documented error codes.  No device work."""
import numpy as np
import pytest

from paper_2310_09204_amd import lib, meshes
from oracle.topology import Topology


def _compare(m):
    h = lib.mesh_analyze(m.vertices, m.triangles)
    t = Topology(m.vertices, m.triangles)
    assert h["n_dofs"] == t.N
    assert np.array_equal(h["q"], t.q.astype(np.int32))
    assert [(int(v), int(j)) for v, j in zip(h["dof_vertex"], h["dof_sector"])] == t.dofs
    return h


@pytest.mark.parametrize("name", ["square", "book", "crossed", "crossed_sym", "bowtie", "disk", "fin"])
def test_sector_analysis_matches_oracle(name):
    if name == "square":
        m = meshes.unit_square(8)
    elif name == "book":
        m = meshes.book(6, (0.0, 75.0, 200.0, 300.0))
    elif name == "crossed":
        m = meshes.crossed(8)
    elif name == "crossed_sym":
        m = meshes.crossed(6, symmetric=True)
    elif name == "bowtie":
        m = meshes.bowtie(5)
    elif name == "disk":
        m = meshes.disk(5)
    else:
        m = meshes.build_mesh([meshes.Panel((0, 0, 0), (0.5, 0, 0), (0, 1, 0), 4, 8),
                               meshes.Panel((0.5, 0, 0), (0.5, 0, 0), (0, 1, 0), 4, 8),
                               meshes.Panel((0.5, 0, 0), (0, 0, 0.5), (0, 1, 0), 4, 8)])
    _compare(m)


def test_random_extruded_layouts_match_oracle():
    rng = np.random.default_rng(3)
    for lay in ("book", "chain", "tree"):
        m, _ = meshes.random_extruded(rng, 4, lay, 5)
        _compare(m)


def test_workload_dof_counts():
    for name, n in (("square16", 225), ("book48", 6721)):
        w = meshes.workload(name)
        assert lib.mesh_analyze(w.mesh.vertices, w.mesh.triangles)["n_dofs"] == n
    m = meshes.crossed(96)
    assert lib.mesh_analyze(m.vertices, m.triangles)["n_dofs"] == 27361


def test_rejections():
    V = np.array([[0., 0, 0], [1, 0, 0], [0, 1, 0], [2, 0, 0], [0, 0, 1]])
    cases = [
        (V, [[0, 1, 3]], "BEM_E_DEGENERATE"),
        (V, [[0, 1, 1]], "BEM_E_DEGENERATE"),
        (V, [[0, 1, 2], [1, 2, 0]], "BEM_E_MESH_NONCONFORMING"),
        (V, [[0, 1, 7]], "BEM_E_INVALID_ARG"),
        (np.array([[0., 0, 0], [0, 0, 1], [1, 0, 0], [2, 0, 0.5]]), [[0, 1, 2], [0, 1, 3]], "BEM_E_MESH_NONCONFORMING"),
        (np.array([[0., 0, 0], [1, 0, 0], [0, 1, 0], [-1, 0, 0.3], [0, -1, 0.2]]), [[0, 1, 2], [0, 3, 4]],
         "BEM_E_POINT_CONTACT"),
        (np.array([[0., 0, 0], [1, 0, 0], [0, 1, 0], [1, 0, 0]]), [[0, 1, 2], [0, 3, 2]], "BEM_E_MESH_NONCONFORMING"),
    ]
    for Vc, T, name in cases:
        with pytest.raises(lib.BemError) as e:
            lib.mesh_analyze(Vc, np.array(T))
        assert e.value.name == name, (T, e.value)
