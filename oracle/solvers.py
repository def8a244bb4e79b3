"""Outer iterations (oracle, test infrastructure).

  preconditioned damped Richardson   x <- x + xi C^{-1} (b - A x)   (Alg. 3)
  optimal damping and rate           xi* = 2/(lmin+lmax),
                                     rho* = 1 - 2/(1+kappa)         (eq. redrate)
  preconditioned CG                  textbook Hestenes-Stiefel (Sec. 3.3)
  flexible CG                        beta = z_{k+1}^T (r_{k+1} - r_k) / z_k^T r_k
                                     (the variant the paper names for a
                                      non-symmetric preconditioner)
Stopping: relative true residual ||b - A x||_2 / ||b||_2 <= rtol, or, for the
paper's protocol (Sec. 4: f = 0, random x0 scaled to ||x0||_A = 1), the energy
norm of the iterate (which is then the error) dropping to <= tol.
"""
from __future__ import annotations

from typing import Callable, Optional

import numpy as np


def _stop_fn(A, b, rtol, energy_tol):
    if energy_tol is not None:
        return lambda x, r: np.sqrt(max(float(x @ (A @ x)), 0.0)) <= energy_tol
    nb = float(np.linalg.norm(b))
    return lambda x, r: float(np.linalg.norm(b - A @ x)) <= rtol * nb


def pcg(A, b, M: Callable, x0=None, rtol=1e-9, maxit=1000, flexible=False,
        energy_tol: Optional[float] = None, record=False):
    """Returns (x, iterations, info).  info holds the CG coefficients
    (alphas, betas) for the Lanczos eigenvalue estimate."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    stop = _stop_fn(A, b, rtol, energy_tol)
    alphas, betas = [], []
    if stop(x, r):
        return x, 0, {"alphas": alphas, "betas": betas}
    z = M(r)
    p = z.copy()
    rz = float(r @ z)
    for k in range(1, maxit + 1):
        q = A @ p
        alpha = rz / float(p @ q)
        x = x + alpha * p
        r_old = r
        r = r - alpha * q
        alphas.append(alpha)
        if stop(x, r):
            return x, k, {"alphas": alphas, "betas": betas}
        z = M(r)
        if flexible:
            beta = float(z @ (r - r_old)) / rz
        else:
            beta = float(r @ z) / rz
        betas.append(beta)
        rz = float(r @ z)
        p = z + beta * p
    return x, maxit, {"alphas": alphas, "betas": betas, "not_converged": True}


def lanczos_extremes(alphas, betas):
    """Extreme Ritz values of C^{-1}A from the CG coefficients: the Lanczos
    tridiagonal has T_kk = 1/a_k + b_{k-1}/a_{k-1}, T_{k,k+1} = sqrt(b_k)/a_k."""
    m = len(alphas)
    if m == 0:
        raise ValueError("no CG steps")
    T = np.zeros((m, m))
    for k in range(m):
        T[k, k] = 1.0 / alphas[k] + (betas[k - 1] / alphas[k - 1] if k > 0 else 0.0)
        if k + 1 < m:
            T[k, k + 1] = T[k + 1, k] = np.sqrt(betas[k]) / alphas[k]
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])


def richardson(A, b, M: Callable, xi: float, x0=None, rtol=1e-9, maxit=100000,
               energy_tol: Optional[float] = None):
    """Alg. 3: x^{k+1} = x^k + xi C^{-1} (b - A x^k).  Returns (x, iterations)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    stop = _stop_fn(A, b, rtol, energy_tol)
    r = b - A @ x
    if stop(x, r):
        return x, 0
    for k in range(1, maxit + 1):
        x = x + xi * M(r)
        r = b - A @ x
        if stop(x, r):
            return x, k
    return x, maxit


def dense_spectrum(A_dense: np.ndarray, Cinv_dense: np.ndarray):
    """(lambda_min, lambda_max) of C^{-1} A by a dense eigen-solve (tiny grids)."""
    ev = np.linalg.eigvals(Cinv_dense @ A_dense).real
    return float(ev.min()), float(ev.max())


def optimal_damping(lmin: float, lmax: float):
    """eq. (redrate): xi* = 2/(lmin+lmax), rho* = 1 - 2/(1+kappa)."""
    kappa = lmax / lmin
    return 2.0 / (lmin + lmax), 1.0 - 2.0 / (1.0 + kappa)


def paper_start(A, seed: int, n: int):
    """Sec. 4 protocol: x0 entries iid U[-1,1] (splitmix64 stands in for the
    unspecified STL engine), rescaled so that ||x0||_A = 1."""
    from seeded_inputs import uniform_pm1
    x = uniform_pm1(seed, n)
    return x / np.sqrt(float(x @ (A @ x)))


def cg_coefficients(A, b, M: Callable, steps: int):
    """Run `steps` PCG steps regardless of convergence (stopping early only on
    an exact breakdown) and return the coefficient lists for lanczos_extremes."""
    x = np.zeros_like(b)
    r = b.copy()
    z = M(r)
    p = z.copy()
    rz = float(r @ z)
    alphas, betas = [], []
    for _ in range(steps):
        q = A @ p
        pq = float(p @ q)
        if pq <= 0.0 or rz <= 0.0:
            break
        alpha = rz / pq
        r = r - alpha * q
        alphas.append(alpha)
        z = M(r)
        rz_new = float(r @ z)
        if rz_new <= 0.0:
            break
        betas.append(rz_new / rz)
        rz = rz_new
        p = z + betas[-1] * p
    return alphas, betas[: max(len(alphas) - 1, 0)]
