"""GPU double-layer potential (Lemma repDL) against the oracle, through the C-ABI."""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_2310_09204_amd import lib, meshes
from oracle.potential import double_layer
from oracle.topology import Topology

pytestmark = pytest.mark.gpu
NEAR = 10


def _targets(m, count, seed, min_dist=0.25):
    # seeded points in a box around the mesh, at least min_dist from every vertex
    rng = np.random.default_rng(seed)
    lo, hi = m.vertices.min(0) - 0.8, m.vertices.max(0) + 0.8
    out = []
    while len(out) < count:
        x = lo + (hi - lo) * rng.random(3)
        if np.linalg.norm(m.vertices - x, axis=1).min() >= min_dist:
            out.append(x)
    return np.array(out)


@pytest.mark.parametrize("name,k", [("square8", 1), ("book6", 3), ("crossed6", 17), ("bowtie5", 2)])
def test_double_layer_matches_oracle(ctx, name, k):
    m = {"square8": meshes.unit_square(8), "book6": meshes.book(6), "crossed6": meshes.crossed(6),
         "bowtie5": meshes.bowtie(5)}[name]
    print("case", name, k, flush=True)
    p = lib.Problem(ctx, m.vertices, m.triangles, near_order=NEAR)
    t = Topology(m.vertices, m.triangles)
    phi = np.random.default_rng(5).standard_normal((k, p.N))
    X = _targets(m, 150, 6)
    Ug = p.double_layer(phi, X)
    Uo = double_layer(m.vertices, m.triangles, np.stack([t.jump_values(ph) for ph in phi]), X)
    assert Ug.shape == (k, len(X))
    assert np.abs(Ug - Uo).max() < 1e-12 * np.abs(Uo).max()


def test_double_layer_edge_cases(ctx):
    m = meshes.unit_square(4)
    p = lib.Problem(ctx, m.vertices, m.triangles, near_order=NEAR)
    phi = np.ones((1, p.N))
    assert p.double_layer(phi, np.zeros((0, 3))).shape == (1, 0)
    with pytest.raises(lib.BemError):
        p.double_layer(phi, np.array([[0.5, 0.5, np.nan]]))
    # repeated calls reuse the per-triangle records and give identical results
    X = np.array([[0.3, 0.4, 0.7], [2.0, -1.0, 0.5]])
    assert np.array_equal(p.double_layer(phi, X), p.double_layer(phi, X))


def test_disk_solution_potential_on_the_axis(ctx):
    # solve the flat-disk problem (g = e_z) on the GPU and evaluate its potential on the axis: first
    # order in h towards the exact potential of the jump -(4/pi) sqrt(1 - r^2)
    zs = np.array([0.5, 1.0, 2.0])
    exact = []
    for z in zs:
        f = lambda r: -(4.0 / math.pi) * math.sqrt(1.0 - r * r) * r / (r * r + z * z) ** 1.5
        exact.append(0.5 * z * integrate.quad(f, 0.0, 1.0, epsabs=1e-14, epsrel=1e-13)[0])
    exact = np.array(exact)
    X = np.stack([np.zeros(3), np.zeros(3), zs], axis=1)
    errs = []
    for rings in (12, 24, 48):
        m = meshes.disk(rings)
        p = lib.Problem(ctx, m.vertices, m.triangles, near_order=NEAR)
        phi, info, rc = p.solve(g=np.array([0.0, 0.0, 1.0]), precond=None, tol=1e-12)
        assert rc == 0
        U = p.double_layer(phi, X)[0]
        errs.append(np.abs(U - exact).max() / np.abs(exact).max())
        p.close()
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.006, errs
