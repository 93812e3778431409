"""CPU FP64 oracle for the hypersingular multiscreen BEM (Averseng, Claeys, Hiptmair 2023).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately unoptimised reference
implementation of what the GPU path computes.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute anything under
``oracle/``.  It shares no code with the HIP path (``paper_2310_09204_amd``): topology,
quadrature tables, pair integrals, matrix assembly, preconditioner and solvers are written here
independently, in numpy and in plain C (``pairs.c``).

Modules
  quadrature   7-point degree-5 triangle rule, Gauss-Legendre rule             (Section 4.3 needs
               integrals over pairs of triangles; the rules themselves are the build's reading)
  topology     generalized vertices (sectors), jump basis, jump coefficients    (Section 4.2,
               eqs. defCurlyHOmega .. defYij; Section 4.3 eqs. defAlphaij, defvarphikij)
  pairs        element-pair integrals of 1/(4 pi |x-y|): 7x7 product rule for disjoint pairs,
               Duffy-regularised rules for coincident / edge / vertex pairs      (Cor. corW)
  assemble     Galerkin matrix W and right-hand side L                          (Section 4.3)
  precond      face / wire-basket / coarse additive Schwarz operator M          (eq. jumpSplit,
               Remark "Bound on the number of PCG iterations")
  solve        dense Cholesky solve, PCG, Lanczos condition estimate
  potential    double-layer potential of a discrete jump at points off the screen (Lemma repDL)
  twod         the method on segment multiscreens in the plane (Section 2, Experiments 1 and 2)

Parity status of each function is stated in its docstring; everything here is pinned by the
``-m "not gpu"`` tests in ``tests/test_oracle_*.py`` except where a docstring says
"parity unpinned".
"""
