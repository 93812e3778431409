"""The problem's internal locality order (vertices and triangles in Morton order of their
positions) is invisible at the C-ABI: every call takes and returns data in the caller's numbering.
A problem assembled with keep_order = 1 (the caller's numbering inside as well) and the default,
renumbered one give the same dof tables exactly and the same W, right-hand side, products, pair
integrals, preconditioner, solutions, jump values and potentials within rounding, on a mesh with
junctions (the sector labels and reference sectors depend on the triangle order), in the whole
pair-matrix path and in panels, and through the device-pointer and no-alloc entry points."""
import numpy as np
import pytest

from paper_2310_09204_amd import lib, meshes

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _shuffled(mesh, seed):
    # a mesh whose vertices and triangles come in a random order (the locality order then differs
    # from the caller's numbering everywhere), with the corner order of each triangle kept
    rng = np.random.default_rng(seed)
    V, T = np.asarray(mesh.vertices), np.asarray(mesh.triangles)
    pv = rng.permutation(V.shape[0])
    inv = np.empty_like(pv)
    inv[pv] = np.arange(pv.size)
    pt = rng.permutation(T.shape[0])
    return V[pv], inv[T[pt]].astype(np.int32), pt


@pytest.mark.parametrize("panels", [0, 512])
def test_renumbered_problem_equals_caller_order(ctx, panels):
    base = meshes.book(12, (0.0, 100.0, 230.0))
    V, T, pt = _shuffled(base, 3)
    print("case order book12 shuffled, panels", panels, flush=True)
    kw = dict(near_order=6, precision=lib.FP32_REFINE, keep_pair_matrix=(panels == 0), pair_panel_rows=panels)
    pk = lib.Problem(ctx, V, T, keep_order=True, **kw)
    pr = lib.Problem(ctx, V, T, **kw)
    try:
        N = pk.N
        assert pr.N == N
        assert pk.info["panels_replanned"] == 0 and pr.info["panels_replanned"] == 0
        dk, dr = pk.dofs(), pr.dofs()
        assert np.array_equal(dk[0], dr[0]) and np.array_equal(dk[1], dr[1])
        Wk, Wr = pk.matrix(), pr.matrix()
        assert _rel(Wr, Wk) < 1e-13
        rows = np.array([0, 5, N // 2, N - 1])
        assert _rel(pr.rows(rows), Wk[rows]) < 1e-13
        assert _rel(pr.matrix(3, 7), Wk[3:10]) < 1e-13
        rng = np.random.default_rng(1)
        g = rng.standard_normal((3, 3))
        g /= np.linalg.norm(g, axis=1, keepdims=True)
        assert _rel(pr.rhs(g), pk.rhs(g)) < 1e-14
        x = rng.standard_normal((5, N))
        assert _rel(pr.matvec(x), pk.matvec(x)) < 1e-13
        assert _rel(pr.matvec(x, fp32=True), pk.matvec(x, fp32=True)) < 1e-6
        xd, yd = lib.DeviceArray(x), lib.DeviceArray(shape=x.shape)
        pr.matvec_noalloc(xd.ptr, x.shape[0], yd.ptr)
        assert _rel(yd.get(), x @ Wk.T) < 1e-13
        xd.close()
        yd.close()
        if panels == 0:
            pairs = rng.integers(0, T.shape[0], (500, 2))
            assert _rel(pr.pair_integrals(pairs), pk.pair_integrals(pairs)) < 1e-13
        # preconditioner from per-triangle inputs in the caller's numbering
        patch = meshes.grid_patches(base, 4)[pt]
        cm, par = meshes.coarse_mesh(base, 4)
        par = par[pt]
        Mk = lib.Preconditioner(pk, patch, cm.vertices, cm.triangles, par)
        Mr = lib.Preconditioner(pr, patch, cm.vertices, cm.triangles, par)
        assert Mk.sizes() == Mr.sizes()
        assert _rel(Mr.apply(x), Mk.apply(x)) < 1e-11
        phik, ik, _ = pk.solve(g=g, precond=Mk, tol=1e-12)
        phir, ir, _ = pr.solve(g=g, precond=Mr, tol=1e-12)
        assert _rel(phir, phik) < 1e-10
        assert all(abs(a["iters"] - b["iters"]) <= 1 for a, b in zip(ir, ik))
        x0 = phik + 1e-3 * rng.standard_normal(phik.shape)
        phi0, i0, _ = pr.solve(g=g, precond=Mr, tol=1e-12, x0=x0)
        assert _rel(phi0, phik) < 1e-10
        dout = lib.DeviceArray(shape=phik.shape)
        pr.solve(g=g, precond=Mr, tol=1e-12, device_out=dout.ptr)
        assert _rel(dout.get(), phir) < 1e-14
        dout.close()
        assert _rel(pr.jump_values(phik[0]), pk.jump_values(phik[0])) < 1e-13
        X = np.array([[0.3, 0.4, 1.7], [-1.2, 0.5, 0.9], [0.1, -0.8, -0.6]])
        assert _rel(pr.double_layer(phik, X), pk.double_layer(phik, X)) < 1e-12
        Mk.close()
        Mr.close()
    finally:
        pk.close()
        pr.close()


def test_served_request_in_caller_order(ctx):
    # the serving loop copies each finished column back in the caller's dof order
    base = meshes.book(12, (0.0, 120.0, 240.0))
    V, T, pt = _shuffled(base, 5)
    patch = meshes.grid_patches(base, 6)[pt]
    cm, par = meshes.coarse_mesh(base, 6)
    par = par[pt]
    g = np.array([[0.0, 0.6, 0.8], [1.0, 0.0, 0.0]])
    print("case order serve", flush=True)
    pk = lib.Problem(ctx, V, T, keep_order=True)
    Mk = lib.Preconditioner(pk, patch, cm.vertices, cm.triangles, par)
    ref, _, _ = pk.solve(g=g, precond=Mk, tol=1e-12)
    Mk.close()
    pk.close()
    srv = lib.Server(ctx, max_inflight=1)
    t = srv.submit(V, T, patch, cm.vertices, cm.triangles, par, g, precision=lib.FP64, tol=1e-12)
    phi, info, rc = srv.poll(t)
    srv.close()
    assert rc == 0
    assert _rel(phi, ref) < 1e-10
