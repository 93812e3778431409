"""Writes tests/golden/crossed96_reference.npz: the oracle's exact discrete solution and
preconditioner data on the crossed-panel workload at h = 1/96 (test fixture).

Calls only `oracle/` (and the seeded input generators of `paper_2310_09204_amd.meshes`, which hold
none of the method's arithmetic).  Nothing here comes from the GPU path.

Workload: crossed panels h = 1/96 (55,296 triangles, 27,361 dofs), 96 seeded guillotine patches,
nested coarse mesh H = 1/8, Neumann data g = unit vectors of seeds 0 and 1 (the first two columns
of the benchmark's workload).  Stored:
  * input_hash: sha256 of the mesh, partition, coarse mesh and g (the test refuses a stale file);
  * phi: Phi* = W^{-1} L by dense Cholesky of the oracle's W (Thm. thmBVP: the discrete solution
    is unique; Thm. lemequivInner: W is SPD), one row per g, canonical dof order;
  * energy: L^T Phi* per column (= Phi*^T W Phi*, the squared energy norm of the reference);
  * pcg_iters: iterations of the oracle's PCG (x0 = 0, ||L - W x|| <= 1e-10 ||L||) with the
    additive Schwarz operator of eq. jumpSplit on this partition, per column;
  * sizes: number of face blocks, wire-basket dofs, coarse dofs;
  * apply_idx, apply_z: z = M r at 4,096 seeded dofs for r = default_rng(4).standard_normal(N).

Run: python tests/golden/make_crossed96_reference.py   (about 10 minutes and 20 GB of host memory)
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
from oracle.solve import cholesky_solve, pcg  # noqa: E402
from oracle.topology import Topology  # noqa: E402

NEAR = 10
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "crossed96_reference.npz")


def input_hash(w):
    h = hashlib.sha256()
    for a in (w.mesh.vertices, w.mesh.triangles, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles,
              w.coarse_of_triangle, w.g):
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode() + str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def main():
    t0 = time.time()
    w = meshes.workload("crossed96", seed=0, k=2)
    m = w.mesh
    t = Topology(m.vertices, m.triangles)
    print("topology %.1fs N=%d" % (time.time() - t0, t.N), flush=True)
    W = assemble(m.vertices, m.triangles, t, NEAR)
    print("assembly %.1fs" % (time.time() - t0), flush=True)
    L = rhs(t, w.g)                                      # N x 2
    phi = cholesky_solve(W, L).T.copy()                  # 2 x N
    energy = np.einsum("kn,nk->k", phi, L)
    print("cholesky %.1fs" % (time.time() - t0), flush=True)
    P = AdditiveSchwarz(W, t, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle)
    print("preconditioner %.1fs faces %d wb %d coarse %d" % (time.time() - t0, len(P.face_sets), len(P.wb),
                                                             P.RH.shape[0]), flush=True)
    iters = []
    for c in range(L.shape[1]):
        _, it, relres, _, _ = pcg(W, L[:, c], P.apply, tol=1e-10)
        iters.append(it)
    print("pcg %.1fs iterations %s" % (time.time() - t0, iters), flush=True)
    r = np.random.default_rng(4).standard_normal(t.N)
    z = P.apply(r)
    idx = np.sort(np.random.default_rng(5).choice(t.N, 4096, replace=False))
    np.savez_compressed(OUT, input_hash=np.array(input_hash(w)), phi=phi, energy=energy,
                        pcg_iters=np.array(iters), sizes=np.array([len(P.face_sets), len(P.wb), P.RH.shape[0]]),
                        apply_idx=idx, apply_z=z[idx])
    print("wrote %s (%.1fs)" % (OUT, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
