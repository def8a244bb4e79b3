"""Pins of the seeded inputs and of the oracle's grid, matrix and exact solver."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

from seeded_inputs import splitmix64, uniform_pm1, ct_levels, workloads
from oracle.grid import Grid
from oracle import exact

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vector():
    want = [int(l, 16) for l in open(os.path.join(GOLD, "splitmix64_seed0.txt")) if l.startswith("0x")]
    got = [int(v) for v in splitmix64(0, 3)]
    assert got == want


def test_uniform_range_and_mean():
    u = uniform_pm1(7, 200000)
    assert u.min() >= -1.0 and u.max() < 1.0
    assert abs(u.mean()) < 0.01 and abs(u.var() - 1.0 / 3.0) < 0.01


def test_ct_layer_levels():
    lv = ct_levels(4, 14, 2)
    assert len(lv) == 84                         # compositions of 6 into 4 parts: C(9,3)
    assert all(sum(l) == 14 and min(l) >= 2 for l in lv)
    assert lv == sorted(lv)
    Ns = [int(np.prod([(1 << x) - 1 for x in l])) for l in lv]
    assert min(Ns) == 6885 and max(Ns) == 11025


def test_workload_sizes():
    w = workloads()
    assert w["c1"].N() == 961 and w["c2"].N() == 248031
    assert w["c3"].N() == 252105 and w["c5"].N() == 8258175
    a = w["c3"].coeff
    assert len(a) == 6 and all(0.1 <= v <= 10.0 for v in a)


@pytest.mark.parametrize("levels,coeff", [((3,), None), ((2, 3), None), ((3, 2, 2), (0.5, 2.0, 3.0)),
                                          ((2, 2, 1, 2), (1.0, 0.1, 10.0, 1.0))])
def test_sine_eigenpairs(levels, coeff):
    """A v_k = lambda_k v_k for the closed-form sine eigenpairs."""
    g = Grid(levels=levels, coeff=coeff)
    A = g.matrix()
    rng = np.random.default_rng(0)
    for _ in range(4):
        k = [int(rng.integers(1, n + 1)) for n in g.n]
        v, lam = g.eigen(k)
        assert np.allclose(A @ v, lam * v, rtol=0, atol=1e-9 * abs(lam) * np.abs(v).max())


def test_matrix_stencil_entries():
    """Diagonal sum_j 2 a_j/h_j^2, off-diagonals -a_j/h_j^2 to interior neighbours."""
    g = Grid(levels=(2, 3), coeff=(2.0, 0.5))
    A = g.matrix().toarray()
    c0, c1 = 2.0 * 16, 0.5 * 64
    assert np.allclose(np.diag(A), 2 * c0 + 2 * c1)
    assert A[0, 1] == -c0 and A[0, 3] == -c1 and A[2, 3] == 0.0   # (3,1)-(1,2) not neighbours
    assert np.allclose(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0


@pytest.mark.parametrize("levels,coeff", [((4,), None), ((3, 4), None), ((2, 3, 2), (0.3, 1.0, 7.0))])
def test_dst_solve_matches_dense_lapack(levels, coeff):
    g = Grid(levels=levels, coeff=coeff)
    f = uniform_pm1(3, g.N)
    x_dense = sla.solve(g.matrix().toarray(), f, assume_a="pos")
    x = exact.solve(g, f)
    assert np.linalg.norm(x - x_dense) <= 1e-13 * np.linalg.norm(x_dense)


def test_dst_solve_residual_large():
    g = Grid(levels=(7, 6, 5))
    f = uniform_pm1(2, g.N)
    x = exact.solve(g, f)
    assert np.linalg.norm(g.matrix() @ x - f) <= 1e-12 * np.linalg.norm(f)


def test_anisotropic_reduction_to_1d():
    """Level (m,1,...,1): the operator is the 1-D one plus 8(d-1) I (Sec. 4.2)."""
    m, d = 5, 4
    g = Grid(levels=(m,) + (1,) * (d - 1))
    g1 = Grid(levels=(m,))
    diff = g.matrix() - g1.matrix()
    assert np.allclose(diff.toarray(), 8.0 * (d - 1) * np.eye(g1.N))
