"""Autograd adjoint backward on the GPU against the oracle gradient and
finite differences."""
from fractions import Fraction

import numpy as np
import pytest
import torch

from seeded_inputs import uniform_pm1, log_uniform_coeff
from oracle.grid import Grid
from oracle import exact, grad as ograd

from gpu_common import DEV, dvec, host, relerr, announce

pytestmark = pytest.mark.gpu

import paper_2110_11211_amd as m


@pytest.mark.parametrize("fdtype", ["fp64", "fp32"])
def test_adjoint_gradients_small(fdtype):
    levels = (3, 3, 2, 3)
    announce("adjoint", levels, fdtype)
    a0 = log_uniform_coeff(77, 4)
    g = Grid(levels=levels, coeff=a0)
    f0 = uniform_pm1(6, g.N)
    f = dvec(f0).requires_grad_(True)
    a = torch.tensor(a0, dtype=torch.float64, requires_grad=True)
    u = m.solve_poisson(f, a, levels, P=6, gamma=Fraction(1, 4), factor_dtype=fdtype)
    J = 0.5 * (u * u).sum()
    J.backward()
    u_ref = exact.solve(g, f0)
    gf_ref, ga_ref = ograd.adjoint_gradient(g, u_ref, u_ref)
    assert relerr(host(u), u_ref) <= 1e-9
    assert relerr(host(f.grad), gf_ref) <= 1e-9
    assert np.allclose(a.grad.numpy(), ga_ref, rtol=1e-8, atol=0)
    # central finite difference in a_0 through the GPU solver itself
    h = 1e-5 * a0[0]
    ap, am = a0.copy(), a0.copy()
    ap[0] += h
    am[0] -= h
    with torch.no_grad():
        up = m.solve_poisson(dvec(f0), torch.tensor(ap), levels, P=6, gamma=Fraction(1, 4))
        um = m.solve_poisson(dvec(f0), torch.tensor(am), levels, P=6, gamma=Fraction(1, 4))
    fd = (0.5 * float((up * up).sum()) - 0.5 * float((um * um).sum())) / (2 * h)
    assert abs(fd - a.grad[0].item()) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("fdtype", ["fp32", "fp64"])
def test_adjoint_full_size_d6(fdtype):
    """The d=6 anisotropic-coefficient workload at full size (7^5 x 15 =
    252,105 unknowns, P = 512, gamma = 1/4, a_j log-uniform): forward solve,
    adjoint backward, gradients against the exact DST-I adjoint."""
    from seeded_inputs import workloads
    w = workloads()["c3"]
    levels = w.levels[0]
    announce("adjoint full", levels, fdtype)
    g = Grid(levels=levels, coeff=w.coeff)
    f0 = w.rhs()
    f = dvec(f0).requires_grad_(True)
    a = torch.tensor(w.coeff, dtype=torch.float64, requires_grad=True)
    u = m.solve_poisson(f, a, levels, P=w.P, gamma=w.gamma, factor_dtype=fdtype)
    J = 0.5 * (u * u).sum()
    J.backward()
    u_ref = exact.solve(g, f0)
    gf_ref, ga_ref = ograd.adjoint_gradient(g, u_ref, u_ref)
    assert relerr(host(u), u_ref) <= 1e-9
    assert relerr(host(f.grad), gf_ref) <= 1e-9
    assert np.allclose(a.grad.numpy(), ga_ref, rtol=1e-8, atol=0)
