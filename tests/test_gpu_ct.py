"""Combination technique on the GPU (Sec. 2, eqs. combi and Pchoice; the
Sec. 4.3 model problem) against the oracle: per-grid solutions against the
exact DST-I solutions, the combination kernel against the oracle's
multilinear combination, and the combined error against the manufactured
solution."""
import numpy as np
import pytest
import torch

from oracle import ct, exact
from oracle.grid import Grid

from gpu_common import DEV, dvec, host, relerr, announce

pytestmark = pytest.mark.gpu

import paper_2110_11211_amd as m


def _rhs(CT):
    return np.concatenate([ct.manufactured(CT.grid_points(g))[1] for g in range(CT.ngrids)])


def test_ct_layout_matches_oracle():
    """Grids, layers, weights and subdomain counts of the binding against the
    oracle's enumeration (eq. combi, eq. Pchoice)."""
    announce("ct layout", 3, 5)
    CT = m.CombinationTechnique(3, 5, phat=2, factor_dtype="fp64")
    ref = ct.ct_grids(3, 5)
    assert CT.levels == [lv for lv, _, _ in ref]
    assert CT.layer == [i for _, i, _ in ref]
    assert CT.weights == [w for _, _, w in ref]
    for g, (lv, i, _) in enumerate(ref):
        assert CT.batch._arr[g].P == min(ct.subdomains_per_grid(3, i, 2), Grid(levels=lv).N)
        assert np.array_equal(CT.grid_points(g), ct.grid_points(Grid(levels=lv)))
    CT.close()


@pytest.mark.parametrize("layout", ["natural", "sfc"])
def test_ct_combine_kernel_against_oracle(layout):
    """Combination of arbitrary grid functions at random points (inside the
    cube, on its corners and on grid nodes) against the oracle combine; in
    curve layout the vector is permuted with each grid's curve order."""
    d, L = 3, 5
    announce("ct combine", d, L, layout)
    CT = m.CombinationTechnique(d, L, phat=1, factor_dtype="fp64", layout=layout)
    rng = np.random.default_rng(3)
    sols = [rng.standard_normal(Grid(levels=lv).N) for lv in CT.levels]
    X = np.concatenate([rng.random((300, d)), np.eye(d), np.zeros((1, d)), np.ones((1, d)),
                        CT.grid_points(0)[:20], CT.grid_points(CT.ngrids - 1)[:20]])
    ref = ct.combine(list(zip(CT.levels, CT.weights)), sols, X)
    u = np.concatenate(sols)
    if layout == "sfc":
        perm = np.concatenate([CT.batch.partition(g)["sfc_index"] + CT.batch.offsets[g]
                               for g in range(CT.ngrids)])
        u = u[perm]
    got = host(CT.evaluate(dvec(u), dvec(X)))
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    CT.close()


def test_ct_hat_reproduced():
    """The level-1 tensor hat is in every grid's space: the combination
    reproduces it to rounding (weights sum to one)."""
    d, L = 4, 5
    announce("ct hat", d, L)
    CT = m.CombinationTechnique(d, L, phat=1, factor_dtype="fp64")
    u = np.concatenate([np.prod(1 - np.abs(2 * CT.grid_points(g) - 1), axis=1) for g in range(CT.ngrids)])
    X = np.random.default_rng(4).random((500, d))
    got = host(CT.evaluate(dvec(u), dvec(X)))
    assert np.abs(got - np.prod(1 - np.abs(2 * X - 1), axis=1)).max() <= 1e-13
    CT.close()


@pytest.mark.parametrize("fdtype", ["fp64", "fp32"])
def test_ct_solve_and_combine_against_exact(fdtype):
    """All grids of the d = 3, L = 5 combination solved in one batch; every
    grid's solution against its exact DST-I solution and the combined values
    against the oracle combination of the exact solutions."""
    d, L = 3, 5
    announce("ct solve", d, L, fdtype)
    CT = m.CombinationTechnique(d, L, phat=2, factor_dtype=fdtype)
    f = _rhs(CT)
    u, info = CT.solve(dvec(f), rtol=1e-11)
    uh = host(u)
    sols = []
    for g, lv in enumerate(CT.levels):
        gr = Grid(levels=lv)
        ex = exact.solve(gr, f[CT.batch.offsets[g]:CT.batch.offsets[g + 1]])
        sols.append(ex)
        assert relerr(uh[CT.batch.offsets[g]:CT.batch.offsets[g + 1]], ex) <= 1e-9, (g, lv)
    X = np.random.default_rng(9).random((400, d))
    ref = ct.combine(list(zip(CT.levels, CT.weights)), sols, X)
    got = host(CT.evaluate(u, dvec(X)))
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
    CT.close()


def test_ct_error_decreases_with_level():
    """The combined GPU solution converges to the manufactured solution with
    the level (d = 2): at least a factor 2.5 per level."""
    d = 2
    X = np.random.default_rng(12).random((400, d)) * 0.98 + 0.01
    uex = ct.manufactured(X)[0]
    errs = []
    for L in range(4, 8):
        announce("ct convergence", d, L)
        CT = m.CombinationTechnique(d, L, phat=2, factor_dtype="fp64")
        u, _ = CT.solve(dvec(_rhs(CT)), rtol=1e-12)
        errs.append(np.abs(host(CT.evaluate(u, dvec(X))) - uex).max())
        CT.close()
    assert all(errs[k] / errs[k + 1] >= 2.5 for k in range(len(errs) - 1)), errs


def test_ct_evaluate_rejects_bad_points():
    CT = m.CombinationTechnique(2, 3, factor_dtype="fp64")
    u = torch.zeros(CT.total_unknowns, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        CT.evaluate(u, torch.zeros((5, 3), dtype=torch.float64, device=DEV))
    with pytest.raises(ValueError):
        CT.evaluate(u[:-1], torch.zeros((5, 2), dtype=torch.float64, device=DEV))
    assert CT.evaluate(u, torch.zeros((0, 2), dtype=torch.float64, device=DEV)).numel() == 0
    CT.close()
