"""GPU iteration counts of the Sec. 4.2 dimension study against the oracle.

Setup of Sec. 4.2: isotropic levels l_j = floor((S + log2 P) / d), S = 8,
q = 2^(S-4) = 16, gamma = 1/2, omega-weighted balanced preconditioner; the
Sec. 4 protocol (b = 0, a random start scaled to ||x0||_A = 1, stop when the
energy norm of the error falls below 1e-8).  For d = 2..6 at sizes the oracle
runs in seconds, on the Z-order and on the Hilbert curve, balanced PCG and
balanced Richardson (with the oracle's damping 2 / (lmin + lmax) from its
Lanczos estimate) take the oracle's iteration counts within one.

The paper's own d >= 2 counts come from plots that were lost; its statement
that the counts level off near 26 (Richardson) and 16 (PCG) for d >= 6 is
context only (parity unpinned): the bench reports the GPU counts beside it."""
from fractions import Fraction

import numpy as np
import pytest

from oracle.grid import Grid
from oracle.schwarz import OracleSchwarz
from oracle import solvers
from seeded_inputs import uniform_pm1

from gpu_common import dvec, announce

import paper_2110_11211_amd as m

pytestmark = pytest.mark.gpu

S_LEVEL = 8
Q = 16
GAMMA = Fraction(1, 2)
# (d, P) with S + log2 P a multiple of d and N / P >= q
CASES = [(2, 16), (3, 16), (4, 16), (5, 4), (6, 16)]


def _levels(d, P):
    return (int((S_LEVEL + int(np.log2(P))) // d),) * d


@pytest.mark.parametrize("curve", ["zorder", "hilbert"])
@pytest.mark.parametrize("d,P", CASES)
def test_dimension_study_counts_match_oracle(d, P, curve):
    lv = _levels(d, P)
    announce("dims", d, P, lv, curve)
    g = Grid(levels=lv)
    O = OracleSchwarz(g, P, GAMMA, q=Q, curve=curve)
    x0 = solvers.paper_start(O.A_nat, 11, g.N)
    zero = np.zeros(g.N)
    it_pcg = solvers.pcg(O.A_nat, zero, O.apply, x0=x0, energy_tol=1e-8)[1]
    a, b = solvers.cg_coefficients(O.A_nat, uniform_pm1(99, g.N), O.apply, 150)
    xi, _ = solvers.optimal_damping(*solvers.lanczos_extremes(a, b))
    it_rich = solvers.richardson(O.A_nat, zero, O.apply, xi, x0=x0, energy_tol=1e-8)[1]
    S = m.SFCSchwarz(levels=lv, P=P, gamma=GAMMA, q=Q, curve=curve, factor_dtype="fp64")
    _, ip = S.solve(dvec(zero), x0=dvec(x0), rtol=1e-8, method="pcg", max_iter=2000, plain_start=True,
                    energy=True)
    _, ir = S.solve(dvec(zero), x0=dvec(x0), rtol=1e-8, method="richardson", xi=xi, max_iter=5000,
                    plain_start=True, energy=True)
    S.close()
    print(f"d={d} P={P} l={lv} {curve}: PCG {ip['iterations']} (oracle {it_pcg}), "
          f"Richardson {ir['iterations']} (oracle {it_rich})", flush=True)
    assert abs(ip["iterations"] - it_pcg) <= 1
    assert abs(ir["iterations"] - it_rich) <= 1


def _golden_dims():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "dims_iterations.txt")
    out = {}
    for ln in open(path):
        if ln.strip() and not ln.startswith("#"):
            d, P, curve, itp, itr, xi = ln.split()
            out[(int(d), int(P), curve)] = (int(itp), int(itr), float(xi))
    return out


@pytest.mark.parametrize("curve", ["zorder", "hilbert"])
def test_dimension_study_d6_P1024_matches_oracle(curve):
    """d = 6, P = 1024 (117,649 unknowns): the counts of the stored oracle run
    (golden file) within one.  The paper reports about 16 (PCG) and 26
    (Richardson) for d >= 6 on its Hilbert curve (context, parity unpinned);
    the oracle gives 15 and 26 there."""
    d, P = 6, 1024
    itp, itr, xi = _golden_dims()[(d, P, curve)]
    lv = _levels(d, P)
    announce("dims golden", d, P, curve)
    g = Grid(levels=lv)
    x0 = solvers.paper_start(g.matrix().tocsr(), 11, g.N)
    zero = np.zeros(g.N)
    S = m.SFCSchwarz(levels=lv, P=P, gamma=GAMMA, q=Q, curve=curve, factor_dtype="fp64")
    _, ip = S.solve(dvec(zero), x0=dvec(x0), rtol=1e-8, method="pcg", max_iter=2000, plain_start=True,
                    energy=True)
    _, ir = S.solve(dvec(zero), x0=dvec(x0), rtol=1e-8, method="richardson", xi=xi, max_iter=5000,
                    plain_start=True, energy=True)
    S.close()
    print(f"d=6 P=1024 {curve}: PCG {ip['iterations']} (oracle {itp}), Richardson {ir['iterations']} "
          f"(oracle {itr})", flush=True)
    assert abs(ip["iterations"] - itp) <= 1
    assert abs(ir["iterations"] - itr) <= 1
