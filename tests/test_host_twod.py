"""Host analysis of segment multiscreens (C-ABI, no device work) against the oracle."""
import numpy as np
import pytest

from paper_2310_09204_amd import lib, meshes
from oracle.twod import Topology2D


@pytest.mark.parametrize("mesh", ["plus", "threefold", "slit", "graded", "tree"])
def test_segments_analysis_matches_oracle(mesh):
    if mesh == "tree":
        # a vertex of degree 5 at uneven angles, one arm bent, segments given in mixed orientation
        V = np.array([[0, 0], [1, 0], [0.3, 0.9], [-0.8, 0.4], [-0.5, -0.7], [0.6, -0.6], [1.5, 0.4], [2.0, 0.0]], float)
        S = np.array([[0, 1], [2, 0], [0, 3], [4, 0], [0, 5], [1, 6], [7, 6]], np.int32)
    else:
        V, S = {"plus": meshes.plus2d(4), "threefold": meshes.threefold2d(3), "slit": meshes.slit2d(3),
                "graded": meshes.plus2d(5, grading=2.0)}[mesh]
    a = lib.mesh_analyze_2d(V, S, coefficients=True)
    t = Topology2D(V, S)
    assert a["n_dofs"] == t.N
    assert np.array_equal(a["q"], t.q)
    assert np.array_equal(a["c"], t.c)


def test_segments_rejected():
    V, S = meshes.slit2d(2)
    with pytest.raises(lib.BemError):
        lib.mesh_analyze_2d(V, np.vstack([S, S[:1]]))            # repeated segment
    with pytest.raises(lib.BemError):
        lib.mesh_analyze_2d(V, np.vstack([S, [[0, 0]]]))         # zero length
    Vb = np.vstack([V, [[-0.5, 0.0]]])
    with pytest.raises(lib.BemError):
        lib.mesh_analyze_2d(Vb, np.vstack([S, [[0, len(Vb) - 1]]]))   # overlaps segment 0 at vertex 0
    with pytest.raises(lib.BemError):
        lib.mesh_analyze_2d(V, np.array([[0, 99]], np.int32))
