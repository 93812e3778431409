"""The golden closed-form values agree with their formulas (guards the fixture file itself)."""
import math
import os

import pins

HERE = os.path.dirname(os.path.abspath(__file__))


def load_golden():
    vals = {}
    with open(os.path.join(HERE, "golden", "closed_forms.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_golden_values():
    g = load_golden()
    assert abs(g["unit_square_coulomb"] - pins.unit_square_coulomb()) < 1e-14
    assert abs(g["disk_energy"] - 8.0 / 3.0) < 1e-15
    assert abs(g["disk_phi_center"] + 2.0 / math.pi) < 1e-15
    for n, key in ((96, "dofs_crossed96"), (192, "dofs_crossed192")):
        assert g[key] == 3 * ((n - 1) ** 2 - (2 * n - 3)) + 9 * (n - 2) + 7
    assert g["dofs_book48"] == 3 * 47 * 47 + 47 * 2
    assert g["dofs_square16"] == 15 * 15


def test_crossed96_reference_is_current_and_solves_the_oracle_system():
    # the stored exact solution of the crossed96 workload (written by make_crossed96_reference.py
    # with the oracle only) belongs to the current input generators, and its residual rows with
    # the oracle's own rows and right-hand side vanish (Phi* = W^{-1} L, Thm. thmBVP)
    import hashlib
    import numpy as np
    from paper_2310_09204_amd import meshes
    from oracle.assemble import W_rows, rhs
    from oracle.topology import Topology
    ref = np.load(os.path.join(HERE, "golden", "crossed96_reference.npz"))
    w = meshes.workload("crossed96", seed=0, k=2)
    h = hashlib.sha256()
    for a in (w.mesh.vertices, w.mesh.triangles, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles,
              w.coarse_of_triangle, w.g):
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode() + str(a.shape).encode())
        h.update(a.tobytes())
    assert str(ref["input_hash"]) == h.hexdigest()
    t = Topology(w.mesh.vertices, w.mesh.triangles)
    L = rhs(t, w.g).T
    phi = ref["phi"]
    assert np.allclose(np.einsum("kn,kn->k", L, phi), ref["energy"], rtol=1e-13)
    rows = np.sort(np.random.default_rng(1).choice(t.N, 16, replace=False))
    Wr = W_rows(w.mesh.vertices, w.mesh.triangles, rows, topo=t, near_order=10)
    res = L[:, rows] - phi @ Wr.T
    assert np.abs(res).max() < 1e-10 * np.abs(L).max()
