"""Serving loop through the C-ABI: results in a concurrent mix equal the same solves alone,
same-geometry requests merge into one block PCG, admission by HBM footprint, eviction."""
import numpy as np
import pytest

from paper_2310_09204_amd import lib, meshes

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
TOLMIX = 1e-10


def small_stream(seed, n):
    return meshes.serving_stream(seed, n, rate=1e3, n_range=(150, 700), k_range=(1, 4), cells_per_patch=6,
                                 reuse=0.5)


def solo(ctx, r):
    prec = lib.FP32_REFINE if r.mixed else lib.FP64
    p = lib.Problem(ctx, r.mesh.vertices, r.mesh.triangles, precision=prec)
    M = lib.Preconditioner(p, r.patch_of_triangle, r.coarse.vertices, r.coarse.triangles, r.coarse_of_triangle,
                           factor_fp32=r.mixed)
    phi, _, rc = p.solve(g=r.g, precond=M, tol=TOLMIX if r.mixed else TOL64, precision=prec)
    assert rc == 0
    # FP64 reference of the same request for the mixed-precision accuracy check
    p64 = lib.Problem(ctx, r.mesh.vertices, r.mesh.triangles)
    M64 = lib.Preconditioner(p64, r.patch_of_triangle, r.coarse.vertices, r.coarse.triangles, r.coarse_of_triangle)
    ref, _, _ = p64.solve(g=r.g, precond=M64, tol=1e-13)
    for h in (M, p, M64, p64):
        h.close()
    return phi, ref


def submit(srv, r):
    return srv.submit(r.mesh.vertices, r.mesh.triangles, r.patch_of_triangle, r.coarse.vertices,
                      r.coarse.triangles, r.coarse_of_triangle, r.g,
                      precision=lib.FP32_REFINE if r.mixed else lib.FP64, tol=TOLMIX if r.mixed else TOL64)


def relerr(a, b):
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))


def test_mix_equals_solo(ctx):
    reqs = small_stream(3, 10)
    print("case serve-mix", [(r.geometry, r.mesh.nt, r.g.shape[0], r.mixed) for r in reqs], flush=True)
    alone = [solo(ctx, r) for r in reqs]
    srv = lib.Server(ctx, max_inflight=3)
    tickets = [submit(srv, r) for r in reqs]
    results, messages = [], []
    for t in tickets:
        results.append(srv.poll(t))
        messages.append(srv.last_message)
    st = srv.stats()
    srv.close()
    assert st["submitted"] == len(reqs) and st["completed"] == len(reqs) and st["rejected"] == 0
    for r, (phi_solo, ref), (phi, info, rc), msg in zip(reqs, alone, results, messages):
        assert rc == 0, msg
        assert phi.shape == phi_solo.shape
        assert all(i["t_total_s"] > 0 and 0 < i["t_start_s"] <= i["t_total_s"] for i in info)
        if r.mixed:
            assert relerr(phi, ref) < 1e-8
        else:
            # same algorithm and tolerance alone and in the mix; column blocks differ only in the
            # summation order of the products
            assert relerr(phi, phi_solo) < 1e-10
            assert relerr(phi, ref) < 1e-10


def test_same_geometry_requests_merge(ctx):
    reqs = small_stream(5, 6)
    big = reqs[0]
    base = reqs[1]
    rng = np.random.default_rng(9)
    same = []
    for j in range(3):
        g = rng.standard_normal((j + 1, 3))
        g /= np.linalg.norm(g, axis=1, keepdims=True)
        same.append(meshes.ServeRequest(0.0, 99, base.mesh, base.patch_of_triangle, base.coarse,
                                        base.coarse_of_triangle, g, False))
    print("case serve-merge", big.mesh.nt, base.mesh.nt, flush=True)
    srv = lib.Server(ctx, max_inflight=1)
    t0 = submit(srv, big)           # occupies the only slot while the next three queue up
    ts = [submit(srv, r) for r in same]
    out0 = srv.poll(t0)
    outs = [srv.poll(t) for t in ts]
    st = srv.stats()
    srv.close()
    assert out0[2] == 0
    assert st["merged_batches"] >= 1
    for r, (phi, info, rc) in zip(same, outs):
        assert rc == 0
        phi_solo, ref = solo(ctx, r)
        assert relerr(phi, ref) < 1e-10


def test_admission_rejects_oversized():
    small = lib.Context(0, hbm_budget_bytes=1 << 20)
    r = small_stream(7, 1)[0]
    srv = lib.Server(small, max_inflight=1)
    with pytest.raises(lib.BemError) as e:
        submit(srv, r)
    assert e.value.name == "BEM_E_ADMISSION"
    assert srv.stats()["rejected"] == 1
    srv.close()
    small.close()


def _book_request(angles, seed):
    m = meshes.book(12, angles)
    cm, par = meshes.coarse_mesh(m, 6)
    g = np.random.default_rng(seed).standard_normal((2, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return meshes.ServeRequest(0.0, seed, m, meshes.grid_patches(m, 6), cm, par, g, True)


def test_eviction_keeps_results_correct():
    # two geometries of equal size; the budget holds one of them (resident matrices plus the
    # transient pair matrix) with 2 % to spare, so every switch of geometry must evict
    a = _book_request((0.0, 120.0, 240.0), 1)
    b = _book_request((0.0, 90.0, 200.0), 2)
    n = lib.mesh_analyze(a.mesh.vertices, a.mesh.triangles)["n_dofs"]
    ld = (n + 63) // 64 * 64
    footprint = ld * n * 12 + 2 * ld * n * 2 + a.mesh.nt * a.mesh.nt * 8
    ctx = lib.Context(0, hbm_budget_bytes=int(1.02 * footprint))
    srv = lib.Server(ctx, max_inflight=1)
    order = [a, b, a, b]
    print("case serve-evict", footprint, n, flush=True)
    outs = [srv.poll(submit(srv, r)) for r in order]   # one at a time
    st = srv.stats()
    srv.close()
    assert st["evictions"] >= 3 and st["cache_hits"] == 0
    for r, (phi, info, rc) in zip(order, outs):
        assert rc == 0
        _, ref = solo(ctx, r)
        assert relerr(phi, ref) < 1e-8
    ctx.close()


def test_served_results_match_oracle(ctx):
    # every column of every served request against the oracle's exact discrete solution of its own
    # geometry (dense Cholesky of the oracle's W, Thm. thmBVP), in the L2 and the energy norm:
    # FP64 requests within 1e-10, mixed-precision ones within 1e-8
    from oracle.assemble import assemble, rhs
    from oracle.solve import cholesky_solve
    from oracle.topology import Topology
    reqs = small_stream(11, 8)
    print("case serve-oracle", [(r.geometry, r.mesh.nt, r.g.shape[0], r.mixed) for r in reqs], flush=True)
    srv = lib.Server(ctx, max_inflight=3)
    tickets = [submit(srv, r) for r in reqs]
    outs = [srv.poll(t) for t in tickets]
    srv.close()
    oracle = {}
    for r, (phi, info, rc) in zip(reqs, outs):
        assert rc == 0
        if r.geometry not in oracle:
            t = Topology(r.mesh.vertices, r.mesh.triangles)
            oracle[r.geometry] = (t, assemble(r.mesh.vertices, r.mesh.triangles, t, 10))
        t, W = oracle[r.geometry]
        xs = cholesky_solve(W, rhs(t, r.g))              # N x k
        e = phi - xs.T
        l2 = np.linalg.norm(e, axis=1) / np.linalg.norm(xs, axis=0)
        en = np.sqrt(np.einsum("kn,nk->k", e, W @ e.T) / np.einsum("nk,nk->k", xs, W @ xs))
        bound = 1e-8 if r.mixed else 1e-10
        assert l2.max() < bound and en.max() < bound, (r.geometry, r.mixed, l2, en)


def test_requests_join_a_running_batch(ctx):
    # continuous batching: one geometry, a 12-column request first, then four more on the same
    # geometry a millisecond apart; they attach to the block PCG that the first one opened (during
    # its assembly or its iterations) and start in free column slots.  Every result equals the
    # request solved alone, within the tolerance.
    import time
    base = _book_request((0.0, 120.0, 240.0), 3)
    rng = np.random.default_rng(21)
    reqs = []
    for k in (12, 3, 2, 1, 2):
        g = rng.standard_normal((k, 3))
        g /= np.linalg.norm(g, axis=1, keepdims=True)
        reqs.append(meshes.ServeRequest(0.0, 7, base.mesh, base.patch_of_triangle, base.coarse,
                                        base.coarse_of_triangle, g, False))
    print("case serve-continuous", base.mesh.nt, [r.g.shape[0] for r in reqs], flush=True)
    srv = lib.Server(ctx, max_inflight=2)
    tickets = []
    for r in reqs:
        tickets.append(submit(srv, r))
        time.sleep(1e-3)
    outs = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) and st["merged_batches"] >= 1 and st["admitted_running"] >= 1, st
    for r, (phi, info, rc) in zip(reqs, outs):
        assert rc == 0 and phi.shape == (r.g.shape[0], phi.shape[1])
        phi_solo, ref = solo(ctx, r)
        assert relerr(phi, phi_solo) < 1e-10 and relerr(phi, ref) < 1e-10
        assert all(i["relres"] <= TOL64 for i in info)
