"""One-level dissection of the dense coarse matrix (halves of the curve,
separator last) against the oracle and against the undissected order.

Any symmetric reordering of A_0 gives the same A_0^{-1} (Sec. 3.1 reasons
the same way for the subdomain matrices), so the dissected coarse solve
must reproduce the oracle's coarse operator F = R_0^T A_0^{-1} R_0 (eq.
restr) to the precision of its FP32 factor and inverse.  The grids here are
small 2-D and 3-D ones on which the dissection is taken (at least 16 coarse
tile rows, both halves two tiles or more, separator at most an eighth); the
8192-unknown coarse matrix of the d=3 workload is dissected as well and is
covered by the full-size parity tests."""
from fractions import Fraction

import numpy as np
import pytest
import torch

from seeded_inputs import uniform_pm1
from oracle.grid import Grid
from oracle.schwarz import OracleSchwarz
from oracle import exact, solvers
from gpu_common import dvec, host, relerr, announce

pytestmark = pytest.mark.gpu

import paper_2110_11211_amd as m

FP32_TOL = 2e-4

CASES = [  # levels, P, gamma, q: 1024 coarse unknowns (16 tile rows) each; both
    # well enough conditioned for the FP32 coarse factor (kappa(A) times the
    # ratio of the largest to the smallest coarse block at most 4096)
    ((6, 6), 256, Fraction(1, 2), 4),
    ((6, 5, 5), 256, Fraction(1, 2), 4),
]


def _solver(levels, P, gamma, q, **kw):
    return m.SFCSchwarz(levels=levels, P=P, gamma=gamma, q=q, factor_dtype="fp32", curve="hilbert", **kw)


@pytest.mark.parametrize("variant", ["additive", "balanced"])
@pytest.mark.parametrize("levels,P,gamma,q", CASES)
def test_split_apply_matches_oracle(levels, P, gamma, q, variant):
    """The dissected coarse solve is taken (sfcdd_info.coarse_split) and the
    application matches the oracle's to the FP32 bar; its difference from
    the application with FP64 coarse factor and inverse (no dissection) is
    within four times that of the undissected FP32 coarse solve."""
    announce("coarse split apply", levels, P, gamma, q, variant)
    g = Grid(levels=levels)
    O = OracleSchwarz(g, P, gamma, q=q, variant=variant, curve="hilbert")
    r = uniform_pm1(41, g.N)
    out = {}
    for name, kw in [("split", {}), ("off", {"coarse_split": "off"}),
                     ("fp64", {"coarse_precision": "fp64", "coarse_split": "off"})]:
        S = _solver(levels, P, gamma, q, variant=variant, **kw)
        split = S.info()["coarse_split"]
        if name == "split":
            assert split[2] > 0 and split[0] >= 2 and split[1] >= 2, split
            assert 64 * sum(split) >= S.info()["N0"] > 64 * (sum(split) - 1)
        else:
            assert split == [0, 0, 0]
        out[name] = host(S.apply(dvec(r)))
        S.close()
        del S
        torch.cuda.empty_cache()
    ref = O.apply(r)
    e_split, e_off = relerr(out["split"], ref), relerr(out["off"], ref)
    d_split = relerr(out["split"], out["fp64"])
    d_off = relerr(out["off"], out["fp64"])
    print(f"coarse split {levels} {variant}: vs oracle {e_split:.2e} (undissected {e_off:.2e}); "
          f"vs FP64 coarse {d_split:.2e} (undissected {d_off:.2e})", flush=True)
    assert e_split <= FP32_TOL
    assert d_split <= max(4.0 * d_off, 1e-9)


@pytest.mark.parametrize("levels,P,gamma,q", CASES)
def test_split_solve(levels, P, gamma, q):
    """Balanced flexible CG with the dissected coarse solve: the oracle's PCG
    iteration count within one, and the exact solution to 1e-8."""
    announce("coarse split solve", levels, P, gamma, q)
    g = Grid(levels=levels)
    O = OracleSchwarz(g, P, gamma, q=q, curve="hilbert")
    f = uniform_pm1(43, g.N)
    _, it_o, _ = solvers.pcg(O.A_nat, f, O.apply, x0=O.balancing_start(f), rtol=1e-10)
    S = _solver(levels, P, gamma, q)
    assert S.info()["coarse_split"][2] > 0
    x, info = S.solve(dvec(f), rtol=1e-10)
    print(f"coarse split solve {levels}: {info['iterations']} iterations (oracle {it_o})", flush=True)
    assert abs(info["iterations"] - it_o) <= 1
    assert relerr(host(x), exact.solve(g, f)) <= 1e-8
    S.close()
    del S
    torch.cuda.empty_cache()


FP64_TOL = 1e-12


@pytest.mark.parametrize("variant", ["additive", "balanced"])
@pytest.mark.parametrize("levels,P,gamma,q", CASES)
def test_split_fp64_matches_oracle(levels, P, gamma, q, variant):
    """With FP64 factors the coarse matrix is dissected as well, and then the
    dissected factorisation, the separator's Schur complement and the block
    inverse are checked to FP64 rounding: the application matches the
    oracle's, and the undissected one, to 1e-12."""
    announce("coarse split fp64", levels, P, gamma, q, variant)
    g = Grid(levels=levels)
    O = OracleSchwarz(g, P, gamma, q=q, variant=variant, curve="hilbert")
    r = uniform_pm1(47, g.N)
    out = {}
    for name, split in [("split", "auto"), ("off", "off")]:
        S = m.SFCSchwarz(levels=levels, P=P, gamma=gamma, q=q, factor_dtype="fp64", curve="hilbert",
                         variant=variant, coarse_split=split)
        got = S.info()["coarse_split"]
        assert (got[2] > 0) if split == "auto" else got == [0, 0, 0], got
        out[name] = host(S.apply(dvec(r)))
        S.close()
        del S
        torch.cuda.empty_cache()
    e = relerr(out["split"], O.apply(r))
    d = relerr(out["split"], out["off"])
    print(f"coarse split fp64 {levels} {variant}: vs oracle {e:.2e}, vs undissected {d:.2e}", flush=True)
    assert e <= FP64_TOL and d <= FP64_TOL
