"""GPU parity of the local elimination orders (the subdomain factors stored as
tile envelopes) against the oracle.

The local solves are direct (Sec. 3.1): A_i^{-1} is the same for every
symmetric reordering of A_i, so the two-level operator must match the
oracle's (dense Cholesky in the subdomain's curve order) whatever order the
library eliminates in.  Bars as in test_gpu_parity: 1e-12 relative with FP64
factors, 2e-4 with FP32 factors.  The cases span every tile-envelope path:
d = 1 (the diagonal order falls back to the curve order), the subdomain that
wraps around the end of the curve (two separate pieces of the grid), ragged
tile rows, subdomains of several tile rows, d = 6, a batch of grids with
different shapes, and the explicit-inverse local solver (always the packed
triangle)."""
from fractions import Fraction

import numpy as np
import pytest

from seeded_inputs import uniform_pm1, workloads
from oracle.grid import Grid
from oracle.schwarz import OracleSchwarz

from gpu_common import dvec, host, relerr, announce

pytestmark = pytest.mark.gpu

import paper_2110_11211_amd as m

ORDERS = ["diagonal", "curve", "dense"]

CASES = [  # levels, P, gamma, curve
    ((9,), 4, Fraction(1, 2), "zorder"),           # d = 1
    ((5, 5), 8, Fraction(1, 4), "hilbert"),
    ((7, 2), 11, Fraction(1, 2), "zorder"),        # ragged subdomains
    ((6, 6), 3, Fraction(1, 2), "hilbert"),        # 2,600 points per subdomain: 41 tile rows
    ((5, 4, 4), 6, Fraction(3, 4), "hilbert"),     # the last subdomain wraps around the curve
    ((3, 3, 3), 4, Fraction(1, 2), "zorder"),
    ((2, 2, 2, 2, 2, 2), 16, Fraction(1, 2), "hilbert"),
]


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("levels,P,gamma,curve", CASES)
def test_apply_matches_oracle_fp64(levels, P, gamma, curve, order):
    announce("local order apply", levels, P, gamma, curve, order)
    g = Grid(levels=levels)
    O = OracleSchwarz(g, P, gamma, curve=curve)
    S = m.SFCSchwarz(levels=levels, P=P, gamma=gamma, curve=curve, factor_dtype="fp64", local_order=order)
    for seed in (5, 6):
        v = uniform_pm1(seed, g.N)
        err = relerr(host(S.apply(dvec(v))), O.apply(v))
        assert err < 1e-12, (seed, err)
    info = S.info()
    assert info["local_order"] == m.LOCAL_ORDER[order]
    S.close()


@pytest.mark.parametrize("order", ["diagonal", "curve"])
def test_apply_matches_oracle_fp32(order):
    levels, P, gamma = (6, 5, 5), 16, Fraction(1, 2)
    announce("local order apply fp32", levels, P, gamma, order)
    g = Grid(levels=levels)
    O = OracleSchwarz(g, P, gamma, curve="hilbert")
    S = m.SFCSchwarz(levels=levels, P=P, gamma=gamma, curve="hilbert", factor_dtype="fp32", local_order=order)
    v = uniform_pm1(7, g.N)
    assert relerr(host(S.apply(dvec(v))), O.apply(v)) < 2e-4
    S.close()


def test_envelope_sizes():
    """The dense order reports the packed triangles (sum_i N_i (N_i + 1) / 2
    entries per sweep); the envelope orders store and read less on a d = 3
    grid, the diagonal order least."""
    levels, P, gamma = (6, 5, 5), 16, Fraction(1, 2)
    announce("envelope sizes", levels, P, gamma)
    got = {}
    for order in ORDERS:
        S = m.SFCSchwarz(levels=levels, P=P, gamma=gamma, curve="hilbert", factor_dtype="fp32", local_order=order)
        got[order] = S.info()
        S.close()
    Ni = m.partition_host(levels=levels, P=P, gamma=gamma)[1]
    nt = (Ni + 63) // 64
    dense = got["dense"]
    assert dense["factor_algo_bytes"] == 4 * int(np.sum(Ni * (Ni + 1) // 2))
    assert dense["factor_bytes"] == 4 * 4096 * int(np.sum(nt * (nt + 1) // 2))
    for order in ("curve", "diagonal"):
        assert got[order]["factor_bytes"] < dense["factor_bytes"]
        assert got[order]["factor_algo_bytes"] < dense["factor_algo_bytes"]
    assert got["diagonal"]["factor_bytes"] < got["curve"]["factor_bytes"]
    print({k: (v["factor_bytes"], v["factor_algo_bytes"]) for k, v in got.items()}, flush=True)


def test_batch_matches_oracle():
    grids = [dict(levels=[5, 5], P=8, gamma=Fraction(1, 4), curve="hilbert"),
             dict(levels=[9], P=4, gamma=Fraction(1, 2)),
             dict(levels=[3, 3, 3], P=4, gamma=Fraction(1, 2))]
    announce("local order batch", grids)
    B = m.SFCSchwarzBatch(grids, factor_dtype="fp64")
    vs, refs = [], []
    for k, gk in enumerate(grids):
        g = Grid(levels=gk["levels"])
        O = OracleSchwarz(g, gk["P"], gk["gamma"], curve=gk.get("curve", "zorder"))
        v = uniform_pm1(20 + k, g.N)
        vs.append(v)
        refs.append(O.apply(v))
    out = host(B.apply(dvec(np.concatenate(vs))))
    off = 0
    for v, ref in zip(vs, refs):
        assert relerr(out[off:off + len(v)], ref) < 1e-12
        off += len(v)
    B.close()


def test_inverse_solver_keeps_dense_triangle():
    levels, P, gamma = (5, 5), 8, Fraction(1, 4)
    announce("local order inverse solver", levels, P, gamma)
    g = Grid(levels=levels)
    O = OracleSchwarz(g, P, gamma, curve="hilbert")
    S = m.SFCSchwarz(levels=levels, P=P, gamma=gamma, curve="hilbert", factor_dtype="fp64",
                     local_solver="inverse", local_order="diagonal")
    v = uniform_pm1(9, g.N)
    assert relerr(host(S.apply(dvec(v))), O.apply(v)) < 1e-12
    assert S.info()["local_order"] == m.LOCAL_ORDER["dense"]
    S.close()


def test_headline_curve_order_envelope():
    """The headline workload with the curve-order envelope (the default
    diagonal order is covered by the c2 iteration test): the oracle's
    iteration count within one and the exact solution."""
    from oracle import exact
    w = workloads()["c2"]
    announce("local order headline curve", w.levels[0], w.P)
    g = Grid(levels=w.levels[0])
    f = w.rhs()
    S = m.SFCSchwarz(levels=w.levels[0], P=w.P, gamma=w.gamma, curve="hilbert", factor_dtype="fp32",
                     local_order="curve")
    x, info = S.solve(dvec(f), rtol=w.rtol, method="fcg", max_iter=200)
    err = relerr(host(x), exact.solve(g, f))
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_hilbert_iterations.txt")
    its = int([ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")][0][0])
    print(f"c2 curve-order envelope: {info['iterations']} iterations (oracle {its}), error {err:.3e}, "
          f"factor bytes {S.info()['factor_bytes']}", flush=True)
    assert abs(info["iterations"] - its) <= 1
    assert err < 5e-9
    S.close()
