"""Adjoint gradient of J(u) = 1/2 ||u||_2^2 with A(a) u = f (oracle, test infra).

With u = A^{-1} f and A symmetric:  lambda = A^{-1} dJ/du = A^{-1} u,
dJ/df = lambda and dJ/da_j = -lambda^T (dA/da_j) u = -(1/h_j^2) lambda^T L_j u,
where L_j is the integer second-difference matrix along dimension j of the
model problem of Sec. 4 (constant diagonal diffusion alpha = diag(a_j)).
"""
from __future__ import annotations

import numpy as np

from .grid import Grid
from . import exact


def adjoint_gradient(g: Grid, u: np.ndarray, dJdu: np.ndarray):
    """(dJ/df, dJ/da) for a given upstream gradient dJ/du (natural order)."""
    lam = exact.solve(g, dJdu)
    ga = np.array([-(g.inv_h2[j]) * float(lam @ (g.second_difference(j) @ u)) for j in range(g.d)])
    return lam, ga


def objective(g: Grid, f: np.ndarray) -> float:
    u = exact.solve(g, f)
    return 0.5 * float(u @ u)
