"""Dense reference solve, preconditioned CG and Lanczos condition estimate (test infrastructure).

The discrete solution Phi* = W^{-1} L is unique (Thm. lemequivInner makes W symmetric positive
definite, Thm. thmBVP).  PCG follows the textbook algorithm the paper's Remark on PCG refers to,
with x0 = 0 and the stopping rule ||L - W x||_2 <= tol ||L||_2 on the unpreconditioned residual.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def cholesky_solve(W, L):
    return sla.cho_solve(sla.cho_factor(W, lower=True), L)


def pcg(W, b, apply_M=None, tol=1e-10, max_iter=10000, x0=None):
    """Returns (x, iterations, relres, alphas, betas).  iterations = number of products with W."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - W @ x if x0 is not None else b.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0, [], []
    z = apply_M(r) if apply_M else r.copy()
    p = z.copy()
    rz = float(r @ z)
    alphas, betas = [], []
    it = 0
    relres = np.linalg.norm(r) / nb
    while it < max_iter and relres > tol:
        q = W @ p
        pq = float(p @ q)
        if not pq > 0.0:
            raise FloatingPointError("PCG breakdown: p.Wp <= 0")
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        it += 1
        alphas.append(alpha)
        relres = np.linalg.norm(r) / nb
        if relres <= tol:
            break
        z = apply_M(r) if apply_M else r.copy()
        rz_new = float(r @ z)
        beta = rz_new / rz
        betas.append(beta)
        rz = rz_new
        p = z + beta * p
    return x, it, relres, alphas, betas


def lanczos_cond(alphas, betas):
    """Extreme eigenvalues of M W from the PCG coefficients (the Lanczos tridiagonal matrix)."""
    m = len(alphas)
    if m == 0:
        return float("nan")
    d = np.zeros(m)
    e = np.zeros(max(m - 1, 0))
    for j in range(m):
        d[j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j < m - 1:
            e[j] = np.sqrt(betas[j]) / alphas[j]
    ev = sla.eigvalsh_tridiagonal(d, e)
    return float(ev[-1] / ev[0])


def spectral_cond(A, B=None):
    """kappa of A (or of B A for SPD B) by a dense symmetric eigen-solve (small problems)."""
    if B is None:
        ev = np.linalg.eigvalsh(A)
    else:
        Lb = np.linalg.cholesky(B)
        ev = np.linalg.eigvalsh(Lb.T @ A @ Lb)
    return float(ev[-1] / ev[0])
