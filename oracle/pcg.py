"""Preconditioned conjugate gradients and the Lanczos condition estimate.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper solves the state system with PCG (Section 2) and estimates the
condition number of the preconditioned operator from the CG coefficients
through the Lanczos connection (Section 5, citing Saad, Iterative Methods
for Sparse Linear Systems, Chapter 6).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla


@dataclasses.dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    converged: bool
    relres: float            # recursive residual norm / ||f||
    alphas: list
    betas: list
    history: list            # recursive relative residual per iteration
    iterates: list | None = None


def pcg(A, f, Minv, tol, maxit=5000, x0=None, keep_iterates=False):
    """Hestenes-Stiefel PCG with Fletcher-Reeves beta.

    Stops at the first k with ||r_k||_2 <= tol ||f||_2 (r the recursively
    updated residual).  Records alpha_k and beta_k for the Lanczos estimate.
    ``A`` and ``Minv`` are callables or matrices on the same space as f.
    """
    matvec = A if callable(A) else (lambda v: A @ v)
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    r = f - matvec(x)
    fn = float(np.linalg.norm(f))
    if fn == 0.0:
        return PCGResult(np.zeros_like(f), 0, True, 0.0, [], [], [])
    z = Minv(r)
    p = z.copy()
    rz = float(r @ z)
    alphas, betas, hist = [], [], []
    its = [x.copy()] if keep_iterates else None
    relres = float(np.linalg.norm(r)) / fn
    if relres <= tol:
        return PCGResult(x, 0, True, relres, alphas, betas, hist, its)
    for k in range(1, maxit + 1):
        q = matvec(p)
        pq = float(p @ q)
        if not np.isfinite(pq) or pq <= 0.0:
            raise FloatingPointError("PCG breakdown: p^T K p <= 0")
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        alphas.append(alpha)
        relres = float(np.linalg.norm(r)) / fn
        hist.append(relres)
        if keep_iterates:
            its.append(x.copy())
        if relres <= tol:
            return PCGResult(x, k, True, relres, alphas, betas, hist, its)
        z = Minv(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        betas.append(beta)
        rz = rz_new
        p = z + beta * p
    return PCGResult(x, maxit, False, relres, alphas, betas, hist, its)


def lanczos_matrix(alphas, betas):
    """Tridiagonal Lanczos matrix T_k built from the CG coefficients:
    T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T_{j,j+1} = sqrt(beta_j)/alpha_j.
    """
    k = len(alphas)
    d = np.empty(k)
    e = np.empty(max(k - 1, 0))
    for j in range(k):
        d[j] = 1.0 / alphas[j]
        if j > 0:
            d[j] += betas[j - 1] / alphas[j - 1]
        if j < k - 1:
            e[j] = np.sqrt(betas[j]) / alphas[j]
    return d, e


def lanczos_condition(alphas, betas):
    """lambda_max(T_k) / lambda_min(T_k) (Saad, Chapter 6)."""
    if len(alphas) == 0:
        return float("nan")
    d, e = lanczos_matrix(alphas, betas)
    w = sla.eigvalsh_tridiagonal(d, e)
    return float(w[-1] / w[0])
