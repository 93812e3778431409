"""GPU assembly parity against the oracle (pair integrals, W, L, jump values), through the C-ABI."""
import math

import numpy as np
import pytest

from paper_2310_09204_amd import lib, meshes
from oracle.assemble import W_rows, assemble, pair_matrix, rhs
from oracle.topology import Topology

pytestmark = pytest.mark.gpu
NEAR = 10


def small_meshes():
    rng = np.random.default_rng(5)
    ext, _ = meshes.random_extruded(rng, 3, "tree", 4)
    return {
        "square8": meshes.unit_square(8),
        "book6": meshes.book(6),
        "crossed6": meshes.crossed(6),
        "bowtie5": meshes.bowtie(5),
        "disk4": meshes.disk(4),
        "extruded": ext,
    }


@pytest.mark.parametrize("name", list(small_meshes()))
def test_pair_integrals_all_pairs(ctx, name):
    m = small_meshes()[name]
    print("case", name, m.nt, flush=True)
    p = lib.Problem(ctx, m.vertices, m.triangles, near_order=NEAR, keep_pair_matrix=True)
    nt = m.nt
    pairs = np.array([[i, j] for i in range(nt) for j in range(nt)], dtype=np.int32)
    Ig = p.pair_integrals(pairs).reshape(nt, nt)
    Io = pair_matrix(m.vertices, m.triangles, NEAR)
    assert np.array_equal(Ig, Ig.T)
    rel = np.abs(Ig - Io) / np.abs(Io)
    assert rel.max() < 1e-12, (name, rel.max())


@pytest.mark.parametrize("name", list(small_meshes()))
def test_matrix_rhs_jumps(ctx, name):
    m = small_meshes()[name]
    print("case", name, m.nt, flush=True)
    t = Topology(m.vertices, m.triangles)
    p = lib.Problem(ctx, m.vertices, m.triangles, near_order=NEAR)
    assert p.N == t.N
    dv, ds = p.dofs()
    assert [(int(a), int(b)) for a, b in zip(dv, ds)] == t.dofs
    Wg = p.matrix()
    Wo = assemble(m.vertices, m.triangles, t, NEAR)
    assert np.array_equal(Wg, Wg.T)                       # mirrored writes: exactly symmetric
    err = np.abs(Wg - Wo).max() / np.abs(Wo).max()
    assert err < 1e-12, (name, err)
    g = np.array([[0.3, -0.5, 0.8], [0.0, 0.0, 1.0]])
    Lg = p.rhs(g)
    Lo = rhs(t, g).T
    assert np.abs(Lg - Lo).max() <= 1e-14 * np.abs(Lo).max()
    phi = np.random.default_rng(1).standard_normal(t.N)
    assert np.allclose(p.jump_values(phi), t.jump_values(phi), rtol=0, atol=1e-13 * np.abs(phi).max())
    # matvec against the FP64 product
    for k in (1, 3, 16, 17):
        x = np.random.default_rng(2 + k).standard_normal((k, t.N))
        y = p.matvec(x)
        assert np.abs(y - x @ Wo).max() <= 1e-12 * np.abs(x @ Wo).max(), k


def test_long_star_general_contraction(ctx):
    # 520 triangles meet at the centre: the first column block's star union exceeds the staged
    # kernel's capacity (512 triangles), so its tiles take the general contraction; the others are
    # staged.  Low near order keeps the oracle's 135k vertex-adjacent pairs quick.
    m = meshes.fan(520)
    order = 4
    print("case fan520", m.nt, flush=True)
    t = Topology(m.vertices, m.triangles)
    p = lib.Problem(ctx, m.vertices, m.triangles, near_order=order)
    Wg = p.matrix()
    Wo = assemble(m.vertices, m.triangles, t, order)
    assert np.array_equal(Wg, Wg.T)
    err = np.abs(Wg - Wo).max() / np.abs(Wo).max()
    assert err < 1e-12, err


@pytest.mark.parametrize("name", ["book6", "crossed6", "extruded"])
def test_panelled_assembly_matches(ctx, name):
    # the pair matrix built and contracted in panels of at most 64 triangle rows gives the same W
    m = small_meshes()[name]
    print("case panels", name, m.nt, flush=True)
    t = Topology(m.vertices, m.triangles)
    p = lib.Problem(ctx, m.vertices, m.triangles, near_order=NEAR, precision=lib.FP32_REFINE, pair_panel_rows=64)
    assert p.info["n_pair_panels"] > (1 if t.N > 64 else 0)
    assert p.info["panels_replanned"] == 0   # laid out from the dof forecast, before the analysis
    Wg = p.matrix()
    Wo = assemble(m.vertices, m.triangles, t, NEAR)
    assert np.array_equal(Wg, Wg.T)
    assert np.abs(Wg - Wo).max() / np.abs(Wo).max() < 1e-12
    full = lib.Problem(ctx, m.vertices, m.triangles, near_order=NEAR)
    assert full.info["n_pair_panels"] == 0
    assert np.abs(Wg - full.matrix()).max() <= 1e-14 * np.abs(Wo).max()
    # the FP32 copy written by the panel contraction
    x = np.random.default_rng(3).standard_normal((2, t.N))
    assert np.allclose(p.matvec(x, fp32=True), x @ Wg.astype(np.float32).astype(np.float64), rtol=1e-5, atol=1e-6 * np.abs(x @ Wg).max())


def test_panelled_long_star(ctx):
    # panels with the general contraction kernel (the centre dof's star holds 520 triangles)
    m = meshes.fan(520)
    print("case panels fan520", m.nt, flush=True)
    t = Topology(m.vertices, m.triangles)
    p = lib.Problem(ctx, m.vertices, m.triangles, near_order=4, pair_panel_rows=64)
    assert p.info["n_pair_panels"] > 1 and p.info["panels_replanned"] == 0
    Wg = p.matrix()
    Wo = assemble(m.vertices, m.triangles, t, 4)
    assert np.array_equal(Wg, Wg.T)
    assert np.abs(Wg - Wo).max() / np.abs(Wo).max() < 1e-12


def test_panelled_book48_rows(ctx):
    w = meshes.workload("book48")
    m = w.mesh
    print("case panels book48", m.nt, flush=True)
    pp = lib.Problem(ctx, m.vertices, m.triangles, near_order=NEAR, pair_panel_rows=3000)
    pf = lib.Problem(ctx, m.vertices, m.triangles, near_order=NEAR)
    assert pp.info["n_pair_panels"] >= 4 and pp.info["panels_replanned"] == 0
    rows = np.random.default_rng(4).choice(pp.N, 24, replace=False)
    a, b = pp.rows(rows), pf.rows(rows)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
    Wp = pp.matrix()
    assert np.array_equal(Wp, Wp.T)


def test_panels_with_unused_vertices_and_without_dofs(ctx):
    # vertices that no triangle uses (no dofs, no rows) in the middle of the numbering leave W as it
    # is, and a mesh whose vertices all lie on the screen's boundary has no dofs and no panels
    m = small_meshes()["book6"]
    V, T = np.asarray(m.vertices), np.asarray(m.triangles)
    k = V.shape[0] // 2
    V2 = np.vstack([V[:k], [[0.31, 0.47, 0.59], [0.13, 0.71, 0.23]], V[k:]])
    T2 = np.where(T >= k, T + 2, T).astype(np.int32)
    print("case panels unused vertices", flush=True)
    ref = lib.Problem(ctx, V, T, near_order=NEAR, pair_panel_rows=64)
    p = lib.Problem(ctx, V2, T2, near_order=NEAR, pair_panel_rows=64)
    assert p.N == ref.N and p.info["panels_replanned"] == 0 and p.info["n_pair_panels"] > 1
    Wr = ref.matrix()
    assert np.abs(p.matrix() - Wr).max() <= 1e-13 * np.abs(Wr).max()
    e = lib.Problem(ctx, np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0]]), np.array([[0, 1, 2]], dtype=np.int32),
                    pair_panel_rows=64)
    assert e.N == 0 and e.info["n_pair_panels"] == 0 and e.info["panels_replanned"] == 0
    for x in (ref, p, e):
        x.close()


def test_concurrent_panel_assemblies(ctx):
    # panel-by-panel assemblies on several threads at once share the context's buffer cache and
    # stream list (each takes a problem stream and an upload stream) and return with their panels
    # queued: each W equals the one assembled alone
    import threading
    ms = small_meshes()
    names = ["book6", "crossed6", "extruded", "square8"]
    print("case concurrent panels", flush=True)
    ref = {}
    for n in names:
        p = lib.Problem(ctx, ms[n].vertices, ms[n].triangles, near_order=NEAR, pair_panel_rows=64)
        ref[n] = p.matrix()
        p.close()
    out, errs = {}, []

    def work(n):
        try:
            for _ in range(2):
                q = lib.Problem(ctx, ms[n].vertices, ms[n].triangles, near_order=NEAR, pair_panel_rows=64)
                out.setdefault(n, []).append(q.matrix())
                q.close()
        except Exception as e:   # reported below, on the test's thread
            errs.append((n, e))

    th = [threading.Thread(target=work, args=(n,)) for n in names]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errs, errs
    for n in names:
        assert all(np.array_equal(Wc, ref[n]) for Wc in out[n]), n


@pytest.mark.parametrize("name", ["book6", "crossed6"])
def test_panels_planned_after_analysis(ctx, name, monkeypatch):
    # the path a mesh takes when its sector analysis numbers the dofs otherwise than the forecast
    # from vertex counts: the first panel's far pass is dropped and the panels are planned again
    m = small_meshes()[name]
    print("case panels replanned", name, m.nt, flush=True)
    t = Topology(m.vertices, m.triangles)
    monkeypatch.setenv("BEM_PANELS_AFTER_ANALYSIS", "1")
    p = lib.Problem(ctx, m.vertices, m.triangles, near_order=NEAR, precision=lib.FP32_REFINE, pair_panel_rows=64)
    monkeypatch.delenv("BEM_PANELS_AFTER_ANALYSIS")
    assert p.info["panels_replanned"] == 1 and p.info["n_pair_panels"] > 1
    Wg = p.matrix()
    Wo = assemble(m.vertices, m.triangles, t, NEAR)
    assert np.array_equal(Wg, Wg.T)
    assert np.abs(Wg - Wo).max() / np.abs(Wo).max() < 1e-12
    q = lib.Problem(ctx, m.vertices, m.triangles, near_order=NEAR, precision=lib.FP32_REFINE, pair_panel_rows=64)
    assert q.info["panels_replanned"] == 0
    assert np.array_equal(q.matrix(), Wg)


def test_book48_sampled_rows(ctx):
    w = meshes.workload("book48")
    m = w.mesh
    p = lib.Problem(ctx, m.vertices, m.triangles, near_order=NEAR)
    assert p.N == 6721
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(p.N, 48, replace=False))
    # include spine dofs (q = 3) explicitly
    dv, ds = p.dofs()
    spine = np.nonzero(np.linalg.norm(m.vertices[dv][:, :2], axis=1) < 1e-12)[0]
    rows = np.unique(np.concatenate([rows, spine[:8]]))
    Wg = p.rows(rows)
    Wo = W_rows(m.vertices, m.triangles, rows, near_order=NEAR)
    scale = np.abs(Wo).max()
    assert np.abs(Wg - Wo).max() < 1e-12 * scale
    # symmetry of the full GPU matrix on the sampled rows
    Wfull = p.matrix()
    assert np.array_equal(Wfull[rows], Wg)
    assert np.array_equal(Wfull, Wfull.T)


def test_crossed96_sampled_rows_and_pairs(ctx):
    m = meshes.crossed(96)
    p = lib.Problem(ctx, m.vertices, m.triangles, near_order=NEAR, keep_pair_matrix=True)
    assert p.N == 27361
    rng = np.random.default_rng(1)
    rows = np.sort(rng.choice(p.N, 24, replace=False))
    dv, ds = p.dofs()
    origin = np.nonzero(np.linalg.norm(m.vertices[dv], axis=1) < 1e-12)[0]
    rows = np.unique(np.concatenate([rows, origin]))
    Wg = p.rows(rows)
    Wo = W_rows(m.vertices, m.triangles, rows, near_order=NEAR)
    assert np.abs(Wg - Wo).max() < 1e-12 * np.abs(Wo).max()
    from oracle.assemble import pair_integrals
    pairs = rng.integers(0, m.nt, size=(4000, 2)).astype(np.int32)
    Ig = p.pair_integrals(pairs)
    Io = pair_integrals(m.vertices, m.triangles, pairs, NEAR)
    assert (np.abs(Ig - Io) / np.abs(Io)).max() < 1e-12


def test_fp32_copy_matches_rounding(ctx):
    m = meshes.unit_square(8)
    p = lib.Problem(ctx, m.vertices, m.triangles, precision=lib.FP32_REFINE, near_order=NEAR)
    W = p.matrix()
    for k in (1, 2, 16, 19):
        x = np.random.default_rng(3 + k).standard_normal((k, p.N))
        y32 = p.matvec(x, fp32=True)
        ref = x.astype(np.float32).astype(np.float64) @ W.astype(np.float32).astype(np.float64)
        assert np.abs(y32 - ref).max() < 1e-5 * np.abs(ref).max(), k


def test_invalid_meshes_rejected_before_device_work(ctx):
    V = np.array([[0., 0, 0], [1, 0, 0], [0, 1, 0], [-1, 0, 0.3], [0, -1, 0.2]])
    with pytest.raises(lib.BemError) as e:
        lib.Problem(ctx, V, np.array([[0, 1, 2], [0, 3, 4]]))
    assert e.value.name == "BEM_E_POINT_CONTACT"
