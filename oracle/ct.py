"""Combination technique (oracle, test infrastructure).

Sec. 2, eq. combi: the sparse-grid solution of level L in d dimensions is
combined from the solutions u_l of the anisotropic full grids of the d layers
|l|_1 = L + (d - 1) - i, i = 0 .. d-1, l_j >= 1, with weights
(-1)^i binom(d-1, i).  Each u_l is a grid function on the interior points of
grid l; it is extended by zero on the boundary and evaluated anywhere by
multilinear interpolation (the piecewise multilinear function of the grid).

Sec. 2, eqs. DOFct and Pchoice: layer i holds binom(L+d-2-i, d-1) grids and
every grid of layer i is split into P = Phat 2^(d-1-i) subdomains.

Sec. 4.3: model problem -Laplace(u) = f on [0,1]^d with the exact solution
u(x) = |x|_2 prod_i sin(pi x_i) (zero on the boundary).
"""
from __future__ import annotations

from math import comb
from typing import List, Tuple

import numpy as np

from seeded_inputs import manufactured  # noqa: F401  (the Sec. 4.3 test problem)

from .grid import Grid


def layer_levels(d: int, total: int) -> List[Tuple[int, ...]]:
    """All level vectors l in N^d with l_j >= 1 and |l|_1 = total, in
    lexicographic order."""
    out: List[Tuple[int, ...]] = []

    def rec(prefix, left, k):
        if k == 1:
            if left >= 1:
                out.append(tuple(prefix + [left]))
            return
        for v in range(1, left - (k - 1) + 1):
            rec(prefix + [v], left - v, k - 1)

    rec([], total, d)
    return out


def ct_grids(d: int, L: int):
    """[(level vector, layer i, weight)] of the combination technique (eq. combi)."""
    out = []
    for i in range(d):
        w = (-1) ** i * comb(d - 1, i)
        for lv in layer_levels(d, L + d - 1 - i):
            out.append((lv, i, float(w)))
    return out


def subdomains_per_grid(d: int, i: int, phat: int) -> int:
    """eq. Pchoice: P = Phat 2^(d-1-i)."""
    return phat * (1 << (d - 1 - i))


def total_subdomains(d: int, L: int, phat: int) -> int:
    """Total number of subdomains over all grids, by the closed form that
    follows eq. Pchoice: Phat/(d-1)! sum_k 2^(d-1-k) prod_{i=1}^{d-1} (L+d-1-k-i)."""
    s = 0
    for k in range(d):
        prod = 1
        for i in range(1, d):
            prod *= (L + d - 1 - k - i)
        s += (1 << (d - 1 - k)) * prod
    f = 1
    for v in range(2, d):
        f *= v
    return phat * s // f


def grid_points(g: Grid) -> np.ndarray:
    """(N, d) coordinates x_j = k_j h_j of the interior points, natural order."""
    h = np.array([1.0 / (n + 1) for n in g.n])
    return g.coords() * h[None, :]


def interpolate(g: Grid, u: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Multilinear interpolation at x (M, d) of the grid function u (natural
    order, zero on the boundary)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    M, d = x.shape
    # padded array with the boundary zeros, axes (n_d+2, ..., n_1+2)
    full = np.zeros([n + 2 for n in reversed(g.n)])
    full[tuple(slice(1, n + 1) for n in reversed(g.n))] = u.reshape([n for n in reversed(g.n)])
    k = np.empty((M, d), dtype=np.int64)
    t = np.empty((M, d))
    for j in range(d):
        s = x[:, j] * (g.n[j] + 1)
        kj = np.clip(np.floor(s).astype(np.int64), 0, g.n[j])
        k[:, j] = kj
        t[:, j] = s - kj
    out = np.zeros(M)
    for corner in range(1 << d):
        w = np.ones(M)
        idx = []
        for j in range(d):
            b = (corner >> j) & 1
            w = w * (t[:, j] if b else 1.0 - t[:, j])
            idx.append(k[:, j] + b)
        out += w * full[tuple(reversed(idx))]
    return out


def combine(levels_weights, solutions, x: np.ndarray) -> np.ndarray:
    """u^(c)(x) = sum_l w_l u_l(x) (eq. combi)."""
    out = np.zeros(np.atleast_2d(x).shape[0])
    for (lv, w), u in zip(levels_weights, solutions):
        out += w * interpolate(Grid(levels=lv), u, x)
    return out
