"""Pin of the oracle's sampled-row checker (CPU only).

`oracle.assemble.W_rows` computes selected rows of W directly from the stars of their dofs
(Section 4.3, eq. eval_a_phiij with Cor. corW); it is the checker of every large-mesh comparison,
where the whole matrix is too large for the host.  Here it is held against the full matrix of
`oracle.assemble.assemble`, which the other oracle pins tie to closed forms, brute force and the
paper's statements, on meshes with every kind of vertex: boundary, panel interior, the book's
spine (q = 3), the crossed axes (q = 4) and origin (q = 8), and an extruded multiscreen with
junctions at random angles.
"""
import numpy as np
import pytest

from paper_2310_09204_amd import meshes
from oracle.assemble import W_rows, assemble
from oracle.topology import Topology

NEAR = 10


def _cases():
    rng = np.random.default_rng(5)
    ext, _ = meshes.random_extruded(rng, 3, "tree", 4)
    return {"book6": meshes.book(6), "crossed6": meshes.crossed(6), "extruded": ext}


@pytest.mark.parametrize("name", list(_cases()))
def test_sampled_rows_equal_full_matrix_rows(name):
    m = _cases()[name]
    t = Topology(m.vertices, m.triangles)
    W = assemble(m.vertices, m.triangles, t, NEAR)
    rng = np.random.default_rng(3)
    rows = rng.choice(t.N, min(t.N, 24), replace=False)
    # every dof at a junction vertex (q >= 3) as well
    junction = [d for d, (v, j) in enumerate(t.dofs) if t.q[v] >= 3]
    rows = np.unique(np.concatenate([rows, np.asarray(junction, dtype=np.int64)])).astype(np.int64)
    R = W_rows(m.vertices, m.triangles, rows, topo=t, near_order=NEAR)
    scale = np.abs(W).max()
    assert R.shape == (len(rows), t.N)
    assert np.abs(R - W[rows]).max() <= 1e-14 * scale, name
    # the rows in any order and with repeats give the same values
    perm = np.concatenate([rows[::-1], rows[:3]])
    R2 = W_rows(m.vertices, m.triangles, perm, topo=t, near_order=NEAR)
    assert np.abs(R2 - W[perm]).max() <= 1e-14 * scale


def test_sampled_rows_catch_a_planted_error():
    # the comparison above is sharp: dropping one triangle of one star changes the row by far more
    # than the tolerance (a mistake in the checker's star walk would not pass unseen)
    m = meshes.crossed(4)
    t = Topology(m.vertices, m.triangles)
    W = assemble(m.vertices, m.triangles, t, NEAR)
    d = next(d for d, (v, j) in enumerate(t.dofs) if t.q[v] == 8)
    full = W_rows(m.vertices, m.triangles, np.array([d]), topo=t, near_order=NEAR)[0]
    # rebuild the same row from all star triangles but one
    from oracle.assemble import _JumpCSR, pair_integrals
    c = _JumpCSR(t)
    tris = c.dof_tri[c.dof_ptr[d]:c.dof_ptr[d + 1]]
    Js = c.dof_J[c.dof_ptr[d]:c.dof_ptr[d + 1]]
    row = np.zeros(t.N)
    for t1, J1 in list(zip(tris, Js))[1:]:
        I = pair_integrals(m.vertices, m.triangles, np.array([[t1, t2] for t2 in range(t.nt)]), NEAR)
        for t2 in range(t.nt):
            for f in range(c.tri_ptr[t2], c.tri_ptr[t2 + 1]):
                row[c.tri_dof[f]] += I[t2] * (J1 @ c.tri_J[f])
    assert np.abs(full - W[d]).max() <= 1e-14 * np.abs(W).max()
    assert np.abs(row - W[d]).max() > 1e-6 * np.abs(W).max()


def test_panel_contraction_equals_full_matrix():
    # the contraction step on its own (panels of rows of I, any dof range), as the CPU baseline times
    # it, adds up to the upper triangle of the full matrix
    from oracle.assemble import I_rows, W_accumulate, _JumpCSR
    m = meshes.crossed(6)
    t = Topology(m.vertices, m.triangles)
    W = assemble(m.vertices, m.triangles, t, NEAR)
    c = _JumpCSR(t)
    U = np.zeros((t.N, t.N))
    half = t.N // 2
    for r0 in range(0, t.nt, 37):
        I = I_rows(m.vertices, m.triangles, r0, min(37, t.nt - r0), NEAR)
        U[:half] += W_accumulate(t, r0, I, 0, half, c)
        U[half:] += W_accumulate(t, r0, I, half, t.N, c)
    iu = np.triu_indices(t.N)
    assert np.abs(U[iu] - W[iu]).max() <= 1e-14 * np.abs(W).max()
    assert np.abs(np.tril(U, -1)).max() == 0.0
