"""The preconditioner of a seeded random (guillotine) partition with a large wire basket, block PCG
columns, start vectors and the non-SPD failure, against the oracle, through the C-ABI.

Workload: crossed panels at h = 1/48 (13,824 triangles, 6,769 dofs), each quadrant cut by seeded
guillotine splits into 16 patches of 10-80 interior vertices: 192 faces and a 2,032-dof wire
basket (patch boundaries, the axes, the screen boundary), nested coarse mesh H = 1/8.  The
additive Schwarz operator is that of eq. jumpSplit; the PCG that of the Remark "Bound on the
number of Preconditioned Conjugate Gradient iterations" (x0 = 0 unless given, unpreconditioned
residual in the stopping rule).
"""
import math

import numpy as np
import pytest

from paper_2310_09204_amd import lib, meshes
from oracle.assemble import assemble, rhs
from oracle.precond import AdditiveSchwarz
from oracle.solve import cholesky_solve, pcg
from oracle.topology import Topology

pytestmark = pytest.mark.gpu
NEAR = 10


def _workload(k=5):
    m = meshes.crossed(48)
    patches = meshes.guillotine_patches(m, np.random.default_rng(0), 2, 16, (10, 80))
    cm, par = meshes.coarse_mesh(m, 6)
    g = np.stack([meshes.unit_g(20 + i) for i in range(k)])
    return meshes.Workload("crossed48-guillotine", m, patches, cm, par, g, "")


@pytest.fixture(scope="module")
def part(ctx):
    w = _workload()
    m = w.mesh
    print("case crossed48 guillotine", m.nt, flush=True)
    t = Topology(m.vertices, m.triangles)
    W = assemble(m.vertices, m.triangles, t, NEAR)
    P = AdditiveSchwarz(W, t, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle)
    L = rhs(t, w.g)                                   # N x k
    xs = cholesky_solve(W, L)                         # N x k
    p64 = lib.Problem(ctx, m.vertices, m.triangles, near_order=NEAR)
    pmx = lib.Problem(ctx, m.vertices, m.triangles, near_order=NEAR, precision=lib.FP32_REFINE)
    M64 = lib.Preconditioner(p64, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle)
    Mmx = lib.Preconditioner(pmx, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle,
                             factor_fp32=True)
    yield w, t, W, P, L, xs, p64, pmx, M64, Mmx
    for h in (Mmx, M64, pmx, p64):
        h.close()


def _errors(phi, xs, W):
    """relative L2 and energy-norm errors of each column of phi [k][N] against xs [N][k]"""
    e = phi - xs.T
    l2 = np.linalg.norm(e, axis=1) / np.linalg.norm(xs, axis=0)
    en = np.sqrt(np.einsum("kn,nk->k", e, W @ e.T) / np.einsum("nk,nk->k", xs, W @ xs))
    return l2, en


def test_partition_sizes_and_apply(part):
    w, t, W, P, L, xs, p64, pmx, M64, Mmx = part
    s = M64.sizes()
    assert s["n_faces"] == len(P.face_sets) == 192
    assert s["n_wb"] == len(P.wb) >= 2000
    assert s["n_coarse"] == P.RH.shape[0]
    assert s["max_face"] == max(len(f) for f in P.face_sets)
    r = np.random.default_rng(4).standard_normal((3, t.N))
    zg = M64.apply(r)
    zo = np.stack([P.apply(ri) for ri in r])
    assert np.abs(zg - zo).max() < 1e-11 * np.abs(zo).max()


def test_partition_pcg_iterations_and_solution(part):
    w, t, W, P, L, xs, p64, pmx, M64, Mmx = part
    for c in range(2):
        _, it_o, _, _, _ = pcg(W, L[:, c], P.apply, tol=1e-10)
        _, info, rc = p64.solve(g=w.g[c], precond=M64, tol=1e-10)
        assert rc == 0 and abs(info[0]["iters"] - it_o) <= 1, (info[0]["iters"], it_o)
    phi, info, rc = p64.solve(g=w.g[:1], precond=M64, tol=1e-13)
    l2, en = _errors(phi, xs[:, :1], W)
    assert l2.max() < 1e-10 and en.max() < 1e-10


@pytest.mark.parametrize("precision", [lib.FP64, lib.FP32_REFINE])
def test_block_pcg_columns_vs_oracle(part, precision):
    # k = 5 right-hand sides in one block PCG: every column against the oracle's exact solution
    w, t, W, P, L, xs, p64, pmx, M64, Mmx = part
    mixed = precision == lib.FP32_REFINE
    p, M = (pmx, Mmx) if mixed else (p64, M64)
    phi, info, rc = p.solve(g=w.g, precond=M, tol=1e-10 if mixed else 1e-13, precision=precision)
    assert rc == 0 and len(info) == 5
    l2, en = _errors(phi, xs, W)
    print("block PCG", "mixed" if mixed else "fp64", l2, en, [i["iters"] for i in info], flush=True)
    bound = 1e-8 if mixed else 1e-10
    assert l2.max() < bound and en.max() < bound


def test_start_vector(part):
    # x0 = Phi* + a perturbation: the oracle's PCG from the same x0 and the GPU's agree in iteration
    # count and solution; x0 = the exact solution needs no iteration
    w, t, W, P, L, xs, p64, pmx, M64, Mmx = part
    x0 = xs[:, 0] + 1e-3 * np.random.default_rng(6).standard_normal(t.N)
    xo, it_o, _, _, _ = pcg(W, L[:, 0], P.apply, tol=1e-10, x0=x0)
    phi, info, rc = p64.solve(g=w.g[:1], precond=M64, tol=1e-10, x0=x0[None, :])
    assert rc == 0 and abs(info[0]["iters"] - it_o) <= 1, (info[0]["iters"], it_o)
    assert np.linalg.norm(phi[0] - xs[:, 0]) / np.linalg.norm(xs[:, 0]) < 1e-8
    phi, info, rc = p64.solve(g=w.g[:1], precond=M64, tol=1e-10, x0=xs[:, 0][None, :])
    assert rc == 0 and info[0]["iters"] == 0
    # mixed precision from a start vector
    phi, info, rc = pmx.solve(g=w.g[:1], precond=Mmx, tol=1e-10, precision=lib.FP32_REFINE, x0=x0[None, :])
    assert rc == 0 and np.linalg.norm(phi[0] - xs[:, 0]) / np.linalg.norm(xs[:, 0]) < 1e-8
    with pytest.raises(ValueError):
        p64.solve(g=w.g[:2], precond=M64, x0=x0[None, :])


def test_indefinite_blocks_rejected(ctx):
    # a diagonal shift below minus the smallest eigenvalue of the blocks makes them indefinite:
    # the set-up reports BEM_E_NOT_SPD (Thm. lemequivInner makes every unshifted block SPD)
    w = meshes.workload("square16")
    m = w.mesh
    p = lib.Problem(ctx, m.vertices, m.triangles, near_order=NEAR)
    W = p.matrix()
    big = 10.0 * np.abs(np.diag(W)).max()
    for wb in ("exact", "diagonal"):
        with pytest.raises(lib.BemError) as e:
            lib.Preconditioner(p, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle,
                               wirebasket=wb, diag_shift=-big)
        assert e.value.name == "BEM_E_NOT_SPD", e.value
    # shift 0 is the default operator; a positive shift gives the operator of W + sigma I blocks
    M0 = lib.Preconditioner(p, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle,
                            diag_shift=0.0)
    M1 = lib.Preconditioner(p, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle)
    r = np.random.default_rng(2).standard_normal((2, p.N))
    assert np.array_equal(M0.apply(r), M1.apply(r))
    t = Topology(m.vertices, m.triangles)
    sigma = 0.1 * np.abs(np.diag(W)).max()
    Ws = assemble(m.vertices, m.triangles, t, NEAR)
    Po = AdditiveSchwarz(Ws, t, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle)
    # the oracle's shifted operator: the same blocks with sigma on their diagonals
    import scipy.linalg as sla
    Po.blocks = [(idx, sla.cho_factor(Ws[np.ix_(idx, idx)] + sigma * np.eye(len(idx)), lower=True))
                 for idx, _ in Po.blocks]
    Po.WH_f = sla.cho_factor(Po.WH + sigma * np.eye(Po.WH.shape[0]), lower=True)
    Ms = lib.Preconditioner(p, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle,
                            diag_shift=sigma)
    zg = Ms.apply(r)
    zo = np.stack([Po.apply(ri) for ri in r])
    assert np.abs(zg - zo).max() < 1e-11 * np.abs(zo).max()
    for h in (Ms, M1, M0, p):
        h.close()
