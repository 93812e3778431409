"""Writes tests/golden/square16_reference.npz and tests/golden/book48_reference.npz: the oracle's
exact discrete solutions, PCG and CG iteration counts and condition-number estimates on the two
small workloads (test and benchmark fixture).

Calls only `oracle/` (and the seeded input generators of `paper_2310_09204_amd.meshes`, which hold
none of the method's arithmetic).  Nothing here comes from the GPU path.

square16: unit square, 16 x 16 cells (512 triangles, 225 dofs), g = (0, 0, 1), 2 x 2 square
          patches (H/h = 8), nested coarse mesh H = 1/2.
book48:   three pages at 0/120/240 degrees on the z-axis, h = 1/48 (13,824 triangles, 6,721 dofs),
          g = unit vectors of seeds 0, 1, 2, 4 x 4 square patches per page (H/h = 12), coarse
          H = 1/4; and the condition-number study of the same book at H/h = 4, 6, 8, 12, 16, 24
          (square patches of H/h cells, nested coarse mesh of the same H).

Stored per workload:
  * input_hash: sha256 of the mesh, partition, coarse mesh and g (consumers refuse a stale file);
  * phi: Phi* = W^{-1} L by dense Cholesky of the oracle's W (Thm. thmBVP; Thm. lemequivInner makes
    W SPD), one row per g, canonical dof order; energy: L^T Phi* per column;
  * pcg_iters / cg_iters: iterations of the oracle's PCG with the additive Schwarz operator of
    eq. jumpSplit, and of plain CG, x0 = 0, ||L - W x|| <= 1e-10 ||L|| (Remark "Bound on the number
    of Preconditioned Conjugate Gradient iterations"), per column;
  * sizes: face blocks, wire-basket dofs, coarse dofs;
  * book48 only, per H/h of the study: kappa_ratio (H/h), kappa_pad (Lanczos estimate of
    kappa(P_ad W) from the PCG on the seed-0 right-hand side at tolerance 1e-12), kappa_iters,
    kappa_sizes (faces, wire basket, coarse); kappa_W: the same estimate for W from plain CG.

Run: python tests/golden/make_small_references.py   (about a minute on 8 cores)
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_2310_09204_amd import meshes  # noqa: E402
from oracle.assemble import assemble, rhs  # noqa: E402
from oracle.precond import AdditiveSchwarz  # noqa: E402
from oracle.solve import cholesky_solve, lanczos_cond, pcg  # noqa: E402
from oracle.topology import Topology  # noqa: E402

NEAR = 10
HERE = os.path.dirname(os.path.abspath(__file__))
KAPPA_RATIOS = (4, 6, 8, 12, 16, 24)


def input_hash(w):
    h = hashlib.sha256()
    for a in (w.mesh.vertices, w.mesh.triangles, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles,
              w.coarse_of_triangle, w.g):
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode() + str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def reference(name, k):
    t0 = time.time()
    w = meshes.workload(name, seed=0, k=k)
    m = w.mesh
    t = Topology(m.vertices, m.triangles)
    W = assemble(m.vertices, m.triangles, t, NEAR)
    print("%s: N=%d assembly %.1fs" % (name, t.N, time.time() - t0), flush=True)
    L = rhs(t, w.g)
    phi = cholesky_solve(W, L).T.copy()
    energy = np.einsum("kn,nk->k", phi, L)
    P = AdditiveSchwarz(W, t, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle)
    pcg_iters, cg_iters = [], []
    for c in range(L.shape[1]):
        pcg_iters.append(pcg(W, L[:, c], P.apply, tol=1e-10)[1])
        cg_iters.append(pcg(W, L[:, c], None, tol=1e-10)[1])
    print("%s: PCG %s CG %s (%.1fs)" % (name, pcg_iters, cg_iters, time.time() - t0), flush=True)
    out = dict(input_hash=np.array(input_hash(w)), phi=phi, energy=energy, pcg_iters=np.array(pcg_iters),
               cg_iters=np.array(cg_iters), sizes=np.array([len(P.face_sets), len(P.wb), P.RH.shape[0]]))
    return w, t, W, L, out


def kappa_study(w, t, W, L):
    """kappa(P_ad W) on the book at fixed h = 1/48 for square patches of H/h cells (Thm. main)."""
    m = w.mesh
    ratios, kp, its, sizes = [], [], [], []
    for r in KAPPA_RATIOS:
        patches = meshes.grid_patches(m, r)
        cm, par = meshes.coarse_mesh(m, r)
        P = AdditiveSchwarz(W, t, patches, cm.vertices, cm.triangles, par)
        _, it, _, a, b = pcg(W, L[:, 0], P.apply, tol=1e-12)
        ratios.append(r)
        kp.append(lanczos_cond(a, b))
        its.append(it)
        sizes.append([len(P.face_sets), len(P.wb), P.RH.shape[0]])
        print("book48 H/h=%d kappa %.3f iterations %d sizes %s" % (r, kp[-1], it, sizes[-1]), flush=True)
    _, it, _, a, b = pcg(W, L[:, 0], None, tol=1e-12)
    return dict(kappa_ratio=np.array(ratios), kappa_pad=np.array(kp), kappa_iters=np.array(its),
                kappa_sizes=np.array(sizes), kappa_W=np.array(lanczos_cond(a, b)))


def main():
    _, _, _, _, out = reference("square16", 1)
    np.savez_compressed(os.path.join(HERE, "square16_reference.npz"), **out)
    w, t, W, L, out = reference("book48", 3)
    out.update(kappa_study(w, t, W, L))
    np.savez_compressed(os.path.join(HERE, "book48_reference.npz"), **out)
    print("wrote square16_reference.npz, book48_reference.npz", flush=True)


if __name__ == "__main__":
    main()
