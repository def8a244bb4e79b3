"""Exact solution A^{-1} f by DST-I diagonalisation (oracle, test infrastructure).

The FD matrix A = sum_j (a_j/h_j^2) L_j of the model problem (Sec. 4) is
diagonalised by the tensor-product sine basis: the discrete sine transform of
type I along every dimension maps A to diag(lambda_k) with
lambda_k = sum_j 4 (a_j/h_j^2) sin^2(k_j pi / (2 (n_j + 1))).  So
x* = IDST(DST(f) / lambda) is the plain definition of the solve's result.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .grid import Grid


def eigenvalues(g: Grid) -> np.ndarray:
    """lambda on the grid, shaped (n_d, ..., n_1) (first coordinate last)."""
    lam = np.zeros([g.n[j] for j in reversed(range(g.d))])
    for j in range(g.d):
        k = np.arange(1, g.n[j] + 1)
        lj = 4.0 * g.c[j] * np.sin(k * np.pi / (2.0 * (g.n[j] + 1))) ** 2
        shape = [1] * g.d
        shape[g.d - 1 - j] = g.n[j]
        lam = lam + lj.reshape(shape)
    return lam


def solve(g: Grid, f: np.ndarray) -> np.ndarray:
    """x* = A^{-1} f, natural order in and out."""
    F = np.asarray(f, dtype=np.float64).reshape([g.n[j] for j in reversed(range(g.d))])
    X = sfft.idstn(sfft.dstn(F, type=1) / eigenvalues(g), type=1)
    return X.reshape(-1)


def extreme_eigenvalues(g: Grid):
    """(lambda_min, lambda_max) of A."""
    lam = eigenvalues(g)
    return float(lam.min()), float(lam.max())
