"""The paper's comparison axes on the GPU (Sec. 4.1, the d = 1 studies:
N = 2^8 P, q = 16): additive against balanced two-level Schwarz with the
three weightings (eqs. addSW, balSW; omega_i, D_i), and the overlap sweep
over gamma.  For d = 1 every space-filling curve is the identity, so the
GPU and the oracle build the same subdomains; iteration counts of FP64 PCG
(flexible CG for the non-symmetric D_i weighting) to a relative recursive
residual of 1e-8 from x0 = 0 must agree within one iteration, and the
qualitative findings of Sec. 4.1 must hold on the GPU."""
from fractions import Fraction

import numpy as np
import pytest

from seeded_inputs import uniform_pm1
from oracle.grid import Grid
from oracle.schwarz import OracleSchwarz
from oracle import solvers

from gpu_common import dvec, announce

pytestmark = pytest.mark.gpu

import paper_2110_11211_amd as m

P = 32
NPTS = [256 * P]
RTOL = 1e-8


def _counts(gamma, variant="balanced", weighting="omega"):
    g = Grid(npts=NPTS)
    b = uniform_pm1(7, g.N)
    flex = weighting == "D"
    O = OracleSchwarz(g, P, gamma, q=16, weighting=weighting, variant=variant)
    it_o = solvers.pcg(O.A_nat, b, O.apply, rtol=RTOL, flexible=flex)[1]
    S = m.SFCSchwarz(npts=NPTS, P=P, gamma=gamma, q=16, weighting=weighting, variant=variant,
                     factor_dtype="fp64")
    _, info = S.solve(dvec(b), rtol=RTOL, method="fcg" if flex else "pcg", plain_start=True,
                      recursive=True)
    S.close()
    return it_o, info["iterations"]


def test_variants_and_weightings_match_oracle():
    """Additive and balanced, each with no weighting, omega_i and D_i: GPU
    counts equal the oracle's (+-1); balanced needs clearly fewer iterations
    than additive, and the balanced weightings coincide."""
    got = {}
    for variant in ("additive", "balanced"):
        for weighting in ("none", "omega", "D"):
            announce("variant", variant, weighting)
            it_o, it_g = _counts(Fraction(1, 2), variant, weighting)
            assert abs(it_g - it_o) <= 1, (variant, weighting, it_o, it_g)
            got[variant, weighting] = it_g
    for w in ("none", "omega", "D"):
        assert got["balanced", w] <= 0.8 * got["additive", w], got
    assert max(got["balanced", w] for w in ("none", "omega", "D")) - \
        min(got["balanced", w] for w in ("none", "omega", "D")) <= 1, got


def test_overlap_sweep_matches_oracle():
    """gamma from 1/5 to 2 (balanced, omega_i): GPU counts equal the
    oracle's (+-1) and fall as the overlap grows."""
    its = []
    for gamma in (Fraction(1, 5), Fraction(1, 2), Fraction(1), Fraction(2)):
        announce("overlap", gamma)
        it_o, it_g = _counts(gamma)
        assert abs(it_g - it_o) <= 1, (gamma, it_o, it_g)
        its.append(it_g)
    assert all(a > b for a, b in zip(its, its[1:])), its


def test_weak_scaling_counts_level_off():
    """Sec. 4.1 weak scaling (N/P = 256 fixed, q = 16, balanced omega_i): the
    GPU counts for P = 64 and 128 equal the oracle's (+-1) and the counts for
    P = 64 .. 512 stay within one iteration of each other."""
    its = {}
    for p in (64, 128, 256, 512):
        announce("weak scaling", p)
        g = Grid(npts=[256 * p])
        b = uniform_pm1(7, g.N)
        S = m.SFCSchwarz(npts=[256 * p], P=p, gamma=Fraction(1, 2), q=16, factor_dtype="fp64")
        _, info = S.solve(dvec(b), rtol=RTOL, method="pcg", plain_start=True, recursive=True)
        S.close()
        its[p] = info["iterations"]
        if p <= 128:
            O = OracleSchwarz(g, p, Fraction(1, 2), q=16)
            it_o = solvers.pcg(O.A_nat, b, O.apply, rtol=RTOL)[1]
            assert abs(its[p] - it_o) <= 1, (p, it_o, its[p])
    assert max(its.values()) - min(its.values()) <= 1, its
