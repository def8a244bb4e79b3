"""Pins of the combination-technique oracle (Sec. 2, eqs. combi, DOFct,
Pchoice; Sec. 4.3 model problem)."""
import os
from math import comb

import numpy as np
import pytest

from oracle import ct, exact
from oracle.grid import Grid

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6])
def test_layer_sizes_and_weights(d):
    """Layer i has binom(L+d-2-i, d-1) grids, and the combination weights sum
    to one over all grids (constants are reproduced)."""
    for L in range(d, d + 6):
        gs = ct.ct_grids(d, L)
        for i in range(d):
            lv = [g for g in gs if g[1] == i]
            assert len(lv) == comb(L + d - 2 - i, d - 1)
            assert all(sum(l) == L + d - 1 - i and min(l) >= 1 for l, _, _ in lv)
        assert abs(sum(w for _, _, w in gs) - 1.0) < 1e-12


def test_total_subdomains_table1():
    """Closed-form total subdomain count against an enumeration of the grids,
    and against the values printed in the paper's Table 1 (L = 20; the d = 6
    cell is read as the closed form at L = 19)."""
    for d in range(1, 7):
        for L in range(d + 1, d + 8):
            tot = sum(ct.subdomains_per_grid(d, i, 4) for _, i, _ in ct.ct_grids(d, L))
            assert tot == ct.total_subdomains(d, L, 4)
    rows = []
    for line in open(os.path.join(GOLD, "ct_subdomains_table1.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append(tuple(map(int, line.split())))
    assert [r[0] for r in rows] == [1, 2, 3, 4, 5, 6]
    for d, L, printed in rows:
        assert ct.total_subdomains(d, L, 1) == printed, (d, L)
    assert ct.total_subdomains(6, 20, 1) != 1754744


@pytest.mark.parametrize("d,L", [(2, 4), (3, 5), (4, 5)])
def test_combination_reproduces_a_common_hat(d, L):
    """The level-1 tensor hat prod_j (1 - |2 x_j - 1|) lies in every grid's
    multilinear space, so interpolation is exact on each grid and the
    combination reproduces it exactly."""
    rng = np.random.default_rng(d)
    X = rng.random((100, d))
    hat = np.prod(1 - np.abs(2 * X - 1), axis=1)
    gs = ct.ct_grids(d, L)
    sols = [np.prod(1 - np.abs(2 * ct.grid_points(Grid(levels=lv)) - 1), axis=1) for lv, _, _ in gs]
    val = ct.combine([(lv, w) for lv, _, w in gs], sols, X)
    assert np.abs(val - hat).max() <= 1e-13


def test_manufactured_solution_is_consistent():
    """f = -Laplace(u) of the manufactured solution, checked by a fourth-order
    central difference of u at random interior points."""
    rng = np.random.default_rng(5)
    for d in (2, 3, 5):
        x = rng.random((20, d)) * 0.8 + 0.1
        u, f = ct.manufactured(x)
        h = 1e-3
        lap = np.zeros(len(x))
        for j in range(d):
            e = np.zeros(d)
            e[j] = h
            up1, _ = ct.manufactured(x + e)
            um1, _ = ct.manufactured(x - e)
            up2, _ = ct.manufactured(x + 2 * e)
            um2, _ = ct.manufactured(x - 2 * e)
            lap += (-up2 + 16 * up1 - 30 * u + 16 * um1 - um2) / (12 * h * h)
        assert np.allclose(-lap, f, rtol=1e-6, atol=1e-6)


def test_sparse_grid_convergence_d2():
    """Combined discrete solutions (exact per grid) converge to the
    manufactured solution at the sparse-grid rate, about a factor 4 per level
    up to the logarithmic term: demand at least 2.5."""
    rng = np.random.default_rng(11)
    X = rng.random((400, 2)) * 0.98 + 0.01
    u, _ = ct.manufactured(X)
    errs = []
    for L in range(3, 8):
        gs = ct.ct_grids(2, L)
        sols = []
        for lv, _, _ in gs:
            g = Grid(levels=lv)
            _, f = ct.manufactured(ct.grid_points(g))
            sols.append(exact.solve(g, f))
        errs.append(np.abs(ct.combine([(lv, w) for lv, _, w in gs], sols, X) - u).max())
    assert all(errs[k] / errs[k + 1] >= 2.5 for k in range(len(errs) - 1)), errs
