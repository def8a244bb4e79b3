"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Bars: index and partition work bit-exact; FP64 operators within 1e-12
(relative 2-norm, well above the ~1e-15 rounding of either side and far
below any plausible indexing or sign error); FP32-factor operators within
2e-4 (tens of FP32 ulps amplified by the local condition numbers, which stay
below ~1e3 at these sizes); solutions within 1e-9 of the exact DST-I solution
(solved to rtol 1e-12)."""
from fractions import Fraction

import numpy as np
import pytest
import torch

from seeded_inputs import uniform_pm1, workloads
from oracle.grid import Grid
from oracle.schwarz import OracleSchwarz
from oracle import exact, solvers
from oracle import grad as ograd
from oracle.sfc import sfc_order

from gpu_common import DEV, dvec, host, relerr, announce

pytestmark = pytest.mark.gpu

import paper_2110_11211_amd as m

FP64_TOL = 1e-12
FP32_TOL = 2e-4

SMALL = [  # levels, P, gamma
    ((5, 5), 8, Fraction(1, 4)),       # the d=2 workload
    ((4, 3), 5, Fraction(1, 2)),
    ((3, 4, 2), 7, Fraction(3, 4)),
    ((6,), 4, Fraction(1, 1)),
    ((3, 3), 3, Fraction(5, 2)),       # every subdomain is the whole grid
    ((4, 4), 6, Fraction(0)),          # no overlap
    ((2, 3, 2, 2), 9, Fraction(1, 3)),
    ((7, 2), 11, Fraction(1, 2)),      # ragged subdomains (N_i not multiples of 64)
    ((3, 1, 1), 7, Fraction(1, 4)),    # P = N, one point per piece, level-1 dimensions
    ((1, 2, 3), 6, Fraction(1, 4)),    # leading level-1 dimension (combination grids)
]


def _solver(levels, P, gamma, **kw):
    return m.SFCSchwarz(levels=levels, P=P, gamma=gamma, **kw)


@pytest.mark.parametrize("curve", ["zorder", "hilbert"])
@pytest.mark.parametrize("levels,P,gamma", SMALL)
def test_sfc_index_and_partition_bit_exact(levels, P, gamma, curve):
    announce("partition", levels, P, gamma, curve)
    S = _solver(levels, P, gamma, curve=curve)
    part = S.partition()
    O = OracleSchwarz(Grid(levels=levels), P, gamma, factor=False, curve=curve)
    assert np.array_equal(part["sfc_index"], O.sfc_index)
    assert np.array_equal(part["ta"], O.ta) and np.array_equal(part["Ni"], O.Ni)
    assert np.array_equal(part["omega"], O.omega) and part["q"] == O.q


@pytest.mark.parametrize("curve", ["zorder", "hilbert"])
@pytest.mark.parametrize("name", ["c2", "c3", "c5"])
def test_sfc_index_full_size(name, curve):
    w = workloads()[name]
    announce("sfc_index", name, curve)
    S = _solver(w.levels[0], w.P, w.gamma, factor_dtype="fp32", curve=curve)
    sfc = S.partition()["sfc_index"]
    ref, _ = sfc_order(Grid(levels=w.levels[0]), curve)
    assert np.array_equal(sfc, ref)
    S.close()
    del S
    torch.cuda.empty_cache()


@pytest.mark.parametrize("levels,P,gamma", SMALL[:4])
def test_matvec(levels, P, gamma):
    announce("matvec", levels, P, gamma)
    g = Grid(levels=levels, coeff=[0.5 + j for j in range(len(levels))])
    S = m.SFCSchwarz(levels=levels, coeff=g.a, P=P, gamma=gamma)
    x = uniform_pm1(3, g.N)
    y = host(S.matvec(dvec(x)))
    assert relerr(y, g.matrix() @ x) <= FP64_TOL


VARIANTS = [("balanced", "omega"), ("additive", "omega"), ("additive", "none"), ("balanced", "none")]


@pytest.mark.parametrize("local", ["cholesky", "inverse"])
@pytest.mark.parametrize("variant,weighting", VARIANTS)
@pytest.mark.parametrize("levels,P,gamma", SMALL)
def test_apply_fp64(levels, P, gamma, variant, weighting, local):
    announce("apply64", levels, P, gamma, variant, weighting, local)
    g = Grid(levels=levels)
    O = OracleSchwarz(g, P, gamma, weighting=weighting, variant=variant)
    S = _solver(levels, P, gamma, weighting=weighting, variant=variant, local_solver=local)
    r = uniform_pm1(7, g.N)
    h = host(S.apply(dvec(r)))
    assert relerr(h, O.apply(r)) <= FP64_TOL


@pytest.mark.parametrize("variant", ["balanced", "additive"])
@pytest.mark.parametrize("levels,P,gamma", SMALL)
def test_apply_fp64_hilbert(levels, P, gamma, variant):
    announce("apply64 hilbert", levels, P, gamma, variant)
    g = Grid(levels=levels)
    O = OracleSchwarz(g, P, gamma, variant=variant, curve="hilbert")
    S = _solver(levels, P, gamma, variant=variant, curve="hilbert")
    r = uniform_pm1(17, g.N)
    h = host(S.apply(dvec(r)))
    assert relerr(h, O.apply(r)) <= FP64_TOL


@pytest.mark.parametrize("variant,weighting", [("deflated", "omega"), ("balanced", "D"), ("additive", "D"),
                                               ("deflated", "D")])
@pytest.mark.parametrize("levels,P,gamma", SMALL)
def test_apply_fp64_deflated_and_D_weights(levels, P, gamma, variant, weighting):
    announce("apply64 variants", levels, P, gamma, variant, weighting)
    g = Grid(levels=levels)
    O = OracleSchwarz(g, P, gamma, weighting=weighting, variant=variant)
    S = _solver(levels, P, gamma, weighting=weighting, variant=variant)
    r = uniform_pm1(19, g.N)
    h = host(S.apply(dvec(r)))
    assert relerr(h, O.apply(r)) <= FP64_TOL


@pytest.mark.parametrize("variant", ["balanced", "deflated"])
def test_fcg_with_D_weights_matches_exact(variant):
    """D_i weights make the preconditioner non-symmetric for gamma = 1/4:
    flexible CG still converges to the exact solution."""
    levels, P, gamma = (5, 4, 3), 12, Fraction(1, 4)
    announce("fcg D", variant)
    g = Grid(levels=levels)
    f = uniform_pm1(10, g.N)
    S = _solver(levels, P, gamma, weighting="D", variant=variant)
    x, info = S.solve(dvec(f), rtol=1e-12, method="fcg", max_iter=500)
    assert relerr(host(x), exact.solve(g, f)) <= 1e-9


def test_pcg_hilbert_iterations_and_solution():
    levels, P, gamma = (5, 4, 4), 16, Fraction(1, 2)
    announce("pcg hilbert")
    g = Grid(levels=levels)
    O = OracleSchwarz(g, P, gamma, curve="hilbert")
    f = uniform_pm1(9, g.N)
    _, it_o, _ = solvers.pcg(O.A_nat, f, O.apply, x0=O.balancing_start(f), rtol=1e-10)
    S = _solver(levels, P, gamma, curve="hilbert")
    x, info = S.solve(dvec(f), rtol=1e-10)
    assert abs(info["iterations"] - it_o) <= 1
    assert relerr(host(x), exact.solve(g, f)) <= 1e-8


@pytest.mark.parametrize("local", ["cholesky", "inverse"])
@pytest.mark.parametrize("levels,P,gamma", SMALL)
def test_apply_fp32_factors(levels, P, gamma, local):
    announce("apply32", levels, P, gamma, local)
    g = Grid(levels=levels)
    O = OracleSchwarz(g, P, gamma)
    S = _solver(levels, P, gamma, factor_dtype="fp32", local_solver=local)
    r = uniform_pm1(8, g.N)
    h = host(S.apply(dvec(r)))
    assert relerr(h, O.apply(r)) <= FP32_TOL


def test_apply_sfc_layout_and_determinism():
    levels, P, gamma = (5, 4, 3), 13, Fraction(1, 2)
    announce("layout", levels)
    g = Grid(levels=levels)
    O = OracleSchwarz(g, P, gamma)
    S = _solver(levels, P, gamma, layout="sfc")
    r = uniform_pm1(9, g.N)
    rs = r[O.sfc_index]
    h1 = host(S.apply(dvec(rs)))
    h2 = host(S.apply(dvec(rs)))
    assert np.array_equal(h1, h2)                     # no atomics: bitwise reproducible
    assert relerr(h1, O.apply_s(rs)) <= FP64_TOL


@pytest.mark.parametrize("plain", [False, True])
def test_pcg_c1_iterations_and_solution(plain):
    """Default: balancing start x0 = F b and one coarse solve per iteration;
    plain: x0 = 0 and the full balanced operator.  Each against the oracle's
    PCG from the same start."""
    w = workloads()["c1"]
    announce("pcg c1", plain)
    g = Grid(levels=w.levels[0])
    O = OracleSchwarz(g, w.P, w.gamma)
    f = w.rhs()
    x0 = None if plain else O.balancing_start(f)
    _, it_o, _ = solvers.pcg(O.A_nat, f, O.apply, x0=x0, rtol=w.rtol)
    S = _solver(w.levels[0], w.P, w.gamma)
    x, info = S.solve(dvec(f), rtol=w.rtol, plain_start=plain)
    assert abs(info["iterations"] - it_o) <= 1
    assert info["rel_residual"] <= w.rtol
    xs = exact.solve(g, f)
    assert relerr(host(x), xs) <= 1e-8


@pytest.mark.parametrize("fdtype,local,method", [("fp64", "cholesky", "pcg"), ("fp64", "inverse", "pcg"),
                                                 ("fp32", "cholesky", "fcg"), ("fp32", "inverse", "fcg")])
@pytest.mark.parametrize("levels,P,gamma", [((5, 5), 8, Fraction(1, 4)), ((4, 3, 3), 10, Fraction(1, 2)),
                                            ((3, 2, 2, 3), 6, Fraction(1, 4))])
def test_solve_matches_exact(levels, P, gamma, fdtype, local, method):
    announce("solve", levels, P, gamma, fdtype, local, method)
    g = Grid(levels=levels)
    f = uniform_pm1(4, g.N)
    S = _solver(levels, P, gamma, factor_dtype=fdtype, local_solver=local)
    x, info = S.solve(dvec(f), rtol=1e-12, method=method)
    assert relerr(host(x), exact.solve(g, f)) <= 1e-9


def test_richardson_fixed_xi_matches_oracle_count():
    levels, P, gamma = (4, 4), 6, Fraction(1, 2)
    announce("richardson")
    g = Grid(levels=levels)
    O = OracleSchwarz(g, P, gamma)
    lmin, lmax = solvers.dense_spectrum(O.A_nat.toarray(), O.dense_preconditioner())
    xi, _ = solvers.optimal_damping(lmin, lmax)
    f = uniform_pm1(5, g.N)
    _, it_o = solvers.richardson(O.A_nat, f, O.apply, xi, rtol=1e-8)
    _, it_b = solvers.richardson(O.A_nat, f, O.apply, xi, x0=O.balancing_start(f), rtol=1e-8)
    S = _solver(levels, P, gamma)
    x, info = S.solve(dvec(f), rtol=1e-8, method="richardson", xi=xi, max_iter=5000, plain_start=True)
    assert abs(info["iterations"] - it_o) <= 1
    xb, infob = S.solve(dvec(f), rtol=1e-8, method="richardson", xi=xi, max_iter=5000)
    assert abs(infob["iterations"] - it_b) <= 1
    x2, info2 = S.solve(dvec(f), rtol=1e-8, method="richardson", xi=0.0, max_iter=5000)
    assert abs(info2["lambda_max"] - lmax) <= 1e-3 * lmax
    assert info2["iterations"] <= 1.5 * it_o + 2
    assert relerr(host(x2), exact.solve(g, f)) <= 1e-6


def test_grad_coeff_matches_oracle():
    levels, coeff = (4, 3, 3), (0.3, 2.0, 5.0)
    announce("grad")
    g = Grid(levels=levels, coeff=coeff)
    u = uniform_pm1(1, g.N)
    lam = uniform_pm1(2, g.N)
    S = m.SFCSchwarz(levels=levels, coeff=coeff, P=4, gamma=Fraction(1, 2))
    ga = S.grad_coeff(dvec(lam), dvec(u))
    ref = [-(g.inv_h2[j]) * float(lam @ (g.second_difference(j) @ u)) for j in range(g.d)]
    assert np.allclose(ga, ref, rtol=1e-12, atol=0)


@pytest.mark.parametrize("fdtype,local", [("fp64", "cholesky"), ("fp32", "cholesky"), ("fp64", "inverse"),
                                          ("fp32", "inverse")])
def test_apply_batched_left_looking_size(fdtype, local):
    """128 subdomains of ~950 points (15 tiles): the batched left-looking
    factorisation path, ragged last tiles."""
    levels, P, gamma = (6, 5, 5), 128, Fraction(1, 2)
    announce("apply-left", fdtype, local)
    g = Grid(levels=levels)
    O = OracleSchwarz(g, P, gamma)
    S = _solver(levels, P, gamma, factor_dtype=fdtype, local_solver=local)
    r = uniform_pm1(12, g.N)
    h = host(S.apply(dvec(r)))
    assert relerr(h, O.apply(r)) <= (FP64_TOL if fdtype == "fp64" else FP32_TOL)


def _coarse_vector(N, P, q, seed):
    """R_0^T c for random c (curve order), from the eq. (restr) blocks."""
    from oracle import partition as part
    c = uniform_pm1(seed, q * P)
    v = np.empty(N)
    for I, (s, sz) in enumerate(part.coarse_blocks(N, P, q)):
        v[s:s + sz] = c[I]
    return v


@pytest.mark.parametrize("name,fdtype", [("c2", "fp32"), ("c2", "fp64"), ("c5", "fp32")])
def test_full_size_solution_and_operator_properties(name, fdtype):
    """Workloads at full size in the benchmark's launch configuration: the
    solve against the exact DST-I solution, and properties of C^{-1} that hold
    at any size: symmetry u^T C^{-1} v = v^T C^{-1} u, and the balanced
    operator's identity on the coarse space, C^{-1} A R_0^T c = R_0^T c."""
    w = workloads()[name]
    announce("full-size", name, fdtype)
    g = Grid(levels=w.levels[0])
    S = _solver(w.levels[0], w.P, w.gamma, factor_dtype=fdtype, layout="sfc")
    f = w.rhs()
    sfc = S.partition()["sfc_index"]
    method = "fcg" if fdtype == "fp32" else "pcg"
    xs_sfc, info = S.solve(dvec(f[sfc]), rtol=1e-12, method=method, max_iter=600)
    x = np.empty(g.N)
    x[sfc] = host(xs_sfc)
    assert relerr(x, exact.solve(g, f)) <= 1e-9
    u = dvec(uniform_pm1(21, g.N))
    v = dvec(uniform_pm1(22, g.N))
    a = float(torch.dot(u, S.apply(v)))
    b = float(torch.dot(v, S.apply(u)))
    assert abs(a - b) <= (1e-12 if fdtype == "fp64" else 1e-5) * abs(a)
    q = S.partition()["q"]
    cv = dvec(_coarse_vector(g.N, w.P, q, 23))
    back = S.apply(S.matvec(cv))
    assert relerr(host(back), host(cv)) <= (1e-10 if fdtype == "fp64" else 1e-5)
    S.close()
    del S
    torch.cuda.empty_cache()


_C2_ORACLES = {}


def _c2_oracle(curve):
    """The oracle's operators of the d=3 workload (factored once per curve)."""
    if curve not in _C2_ORACLES:
        w = workloads()["c2"]
        _C2_ORACLES.clear()
        _C2_ORACLES[curve] = OracleSchwarz(Grid(levels=w.levels[0]), w.P, w.gamma, curve=curve)
    return _C2_ORACLES[curve]


def _kappa(levels):
    """Condition number of the FD matrix from its closed-form extreme
    eigenvalues sum_j 4 (n_j+1)^2 sin^2(k pi / (2 (n_j+1))), k = 1 and n_j."""
    n = np.array([(1 << l) - 1 for l in levels], dtype=np.float64)
    t = np.pi / (2.0 * (n + 1))
    return float(np.sum((n + 1) ** 2 * np.cos(t) ** 2) / np.sum((n + 1) ** 2 * np.sin(t) ** 2))


@pytest.mark.parametrize("curve,fdtype", [("zorder", "fp64"), ("hilbert", "fp64"), ("hilbert", "fp32")])
def test_full_size_apply_c2_matches_oracle(curve, fdtype):
    """One preconditioner application at the d=3 workload's full size (256
    subdomains of ~1937 points) against the oracle, in the default launch
    configuration (tile envelopes in the diagonal order, unit block-lower
    substitution, 16 waves).  FP32 bound: the subdomain
    matrices are principal submatrices of A (kappa(A_i) <= kappa(A), about
    2.9e3 here) and their entries are exact in FP32, so an FP32 Cholesky solve
    errs by a small multiple of kappa(A) * 2^-24; the bar is 4 kappa(A) 2^-24
    (7e-4), the measured error is printed."""
    w = workloads()["c2"]
    announce("full-size apply c2", curve, fdtype)
    O = _c2_oracle(curve)
    S = _solver(w.levels[0], w.P, w.gamma, factor_dtype=fdtype, curve=curve)
    r = uniform_pm1(31, O.N)
    e = relerr(host(S.apply(dvec(r))), O.apply(r))
    tol = FP64_TOL if fdtype == "fp64" else 4.0 * _kappa(w.levels[0]) * 2.0 ** -24
    print(f"c2 apply {curve} {fdtype}: relative error {e:.3e} (bar {tol:.1e})", flush=True)
    assert e <= tol
    S.close()
    del S
    torch.cuda.empty_cache()


def _golden_c2_iterations():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_hilbert_iterations.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    its, res, err = rows[0]
    return int(its), float(res), float(err)


@pytest.mark.parametrize("fdtype", ["fp32", "fp64"])
def test_c2_iteration_count_matches_oracle(fdtype):
    """The benchmark's solve (Hilbert curve, balancing start, rtol 1e-9; FP32
    factors with flexible CG, FP64 factors with PCG) takes the oracle's PCG
    iteration count within one, and reaches the oracle's error against the
    exact solution (golden file written by the oracle's script)."""
    w = workloads()["c2"]
    announce("c2 iterations", fdtype)
    its, _, err_o = _golden_c2_iterations()
    g = Grid(levels=w.levels[0])
    f = w.rhs()
    S = _solver(w.levels[0], w.P, w.gamma, factor_dtype=fdtype, curve="hilbert")
    x, info = S.solve(dvec(f), rtol=w.rtol, method="fcg" if fdtype == "fp32" else "pcg", max_iter=200)
    err = relerr(host(x), exact.solve(g, f))
    print(f"c2 {fdtype}: {info['iterations']} iterations (oracle {its}), residual "
          f"{info['rel_residual']:.3e}, error {err:.3e} (oracle {err_o:.3e})", flush=True)
    assert abs(info["iterations"] - its) <= 1
    assert info["rel_residual"] <= w.rtol
    assert err <= 2.0 * err_o
    S.close()
    del S
    torch.cuda.empty_cache()


def test_batch_heterogeneous_grids_match_single_grid_oracle():
    """A batch of grids of different dimension, size, coefficients, P, gamma
    and q: every grid's block of the batched operator equals the oracle of
    that grid alone, and the batched solve equals each grid's exact solution."""
    grids = [dict(levels=(4, 3), P=5, gamma=Fraction(1, 2)),
             dict(levels=(3, 2, 3), P=7, gamma=Fraction(1, 4), coeff=(0.5, 2.0, 1.5)),
             dict(levels=(5,), P=3, gamma=Fraction(1, 1), q=4),
             dict(levels=(2, 2, 2, 3), P=4, gamma=Fraction(3, 4))]
    announce("batch heterogeneous")
    for fdtype, method in (("fp64", "pcg"), ("fp32", "fcg")):
        S = m.SFCSchwarzBatch(grids, factor_dtype=fdtype)
        rhs, refs_apply, refs_x = [], [], []
        for k, gk in enumerate(grids):
            g = Grid(levels=gk["levels"], coeff=gk.get("coeff"))
            O = OracleSchwarz(g, gk["P"], gk["gamma"], q=gk.get("q"))
            part = S.partition(k)
            assert np.array_equal(part["sfc_index"], O.sfc_index)
            assert np.array_equal(part["ta"], O.ta) and np.array_equal(part["Ni"], O.Ni)
            r = uniform_pm1(40 + k, g.N)
            rhs.append(r)
            refs_apply.append(O.apply(r))
            refs_x.append(exact.solve(g, r))
        rb = dvec(np.concatenate(rhs))
        h = S.split(host(S.apply(rb)))
        for k in range(len(grids)):
            assert relerr(h[k], refs_apply[k]) <= (FP64_TOL if fdtype == "fp64" else FP32_TOL)
        x, info = S.solve(rb, rtol=1e-12, method=method)
        xs = S.split(host(x))
        for k in range(len(grids)):
            assert relerr(xs[k], refs_x[k]) <= 1e-9
        its, res = S.batch_stats()
        assert max(res) <= 1e-12 and info["iterations"] == max(its)


@pytest.mark.parametrize("fdtype,method", [("fp32", "fcg"), ("fp64", "pcg")])
def test_batch_ct_layer_84_grids(fdtype, method):
    """The d=4 combination-technique layer |l|_1 = 14, l_j >= 2 (84 grids of
    6,885 .. 11,025 points, P = 16 each, gamma = 1/4) solved as one batch:
    each grid's solution matches its exact DST-I solution and its iteration
    count equals that of the same grid solved alone."""
    w = workloads()["c4"]
    announce("batch ct", fdtype)
    grids = [dict(levels=lv, P=w.P, gamma=w.gamma) for lv in w.levels]
    S = m.SFCSchwarzBatch(grids, factor_dtype=fdtype)
    S.autotune(3)
    f = np.concatenate([w.rhs(g) for g in range(len(w.levels))])
    x, info = S.solve(dvec(f), rtol=1e-12, method=method, max_iter=400)
    xs = S.split(host(x))
    its, _ = S.batch_stats()
    for g in range(len(w.levels)):
        ref = exact.solve(Grid(levels=w.levels[g]), w.rhs(g))
        assert relerr(xs[g], ref) <= 1e-9, g
    # A single grid factors its coarse matrix with the split-K schedule, a
    # batch with the batched one: the coarse factors round differently, which
    # can move the step that crosses rtol = 1e-12 by one.
    for g in (0, 41, 83):
        Sg = _solver(w.levels[g], w.P, w.gamma, factor_dtype=fdtype)
        _, ig = Sg.solve(dvec(w.rhs(g)), rtol=1e-12, method=method, max_iter=400)
        assert abs(ig["iterations"] - its[g]) <= (1 if fdtype == "fp64" else 2), g


def test_stagnation_status_and_recursive_criterion():
    """A (14, 1) grid (16383 points along x_1): the FP64 rounding floor of the
    true relative residual (about eps ||A|| ||x|| / ||b||, 4e-11 for this
    right-hand side in the oracle's FP64 PCG) lies above 1e-12.
    The verified criterion stops there with ESTAGNATED and an accurate x; the
    recursive criterion of the paper's algorithms reaches rtol."""
    levels = (14, 1)
    announce("stagnation", levels)
    g = Grid(levels=levels)
    f0 = uniform_pm1(31, g.N)
    ex = exact.solve(g, f0)
    S = m.SFCSchwarz(levels=levels, P=128, gamma=Fraction(1, 4), factor_dtype="fp32")
    with pytest.raises(m.SfcddError) as e:
        S.solve(dvec(f0), rtol=1e-12, method="fcg", max_iter=400)
    assert e.value.status == m.ESTAGNATED
    x, info = S.solve(dvec(f0), rtol=1e-12, method="fcg", max_iter=400, check=False)
    assert info["status"] == m.ESTAGNATED and info["iterations"] < 400
    assert relerr(host(x), ex) <= 1e-9
    x2, info2 = S.solve(dvec(f0), rtol=1e-12, method="fcg", max_iter=400, recursive=True)
    assert info2["status"] == m.OK and info2["rel_residual"] <= 1e-12
    assert relerr(host(x2), ex) <= 1e-9
    S.close()


def test_autotune_choice_kept_per_shape():
    """The tuner's choice is kept per launch shape: a second context of the
    same shape gets the same wave count and time without timing again; a
    negative repeat count times again; the solve is unchanged either way."""
    announce("autotune cache")
    kw = dict(levels=(5, 5), P=8, gamma=Fraction(1, 4), factor_dtype="fp32")
    S1 = m.SFCSchwarz(**kw)
    t1 = S1.autotune(2)
    w1 = S1.info()["trsv_waves"]
    S1.close()
    S2 = m.SFCSchwarz(**kw)
    t2 = S2.autotune(2)
    assert S2.info()["trsv_waves"] == w1 and t2 == t1
    t3 = S2.autotune(-2)
    assert t3 > 0 and S2.info()["trsv_waves"] in (4, 8, 16)
    g = Grid(levels=(5, 5))
    f0 = uniform_pm1(1, g.N)
    x, _ = S2.solve(dvec(f0), rtol=1e-12, method="fcg")
    assert relerr(host(x), exact.solve(g, f0)) <= 1e-9
    S2.close()


@pytest.mark.parametrize("fdtype", ["fp32", "fp64"])
def test_tune_launch_shapes_keeps_parity(fdtype):
    """sfcdd_tune over all launch shapes (substitution waves, SpMV points and
    window, factorisation rows and column pairing): the choices lie in the
    candidate sets, the context is left set up with the winning factorisation
    shape and still matches the oracle, and a second context of the same shape
    starts from the recorded shapes and gets the recorded times without timing."""
    levels, P, gamma = (6, 5, 5), 128, Fraction(1, 2)
    announce("tune", fdtype)
    kw = dict(levels=levels, P=P, gamma=gamma, factor_dtype=fdtype, curve="hilbert")
    S1 = m.SFCSchwarz(**kw)
    rep = S1.tune("all", -2)
    print(f"tuning {fdtype}: {rep}", flush=True)
    assert rep["tuned"] == 7
    assert rep["trsv_waves"] in (4, 8, 16)
    assert rep["spmv_points"] in (1, 2, 4) and rep["spmv_window"] == 256 * rep["spmv_points"]
    assert rep["factor_pair"] in (0, 1)
    # rows 1: the light kernel, one column per step
    assert rep["factor_rows"] in ((1, 2, 3, 4) if fdtype == "fp32" else ((1, 2, 3) if rep["factor_pair"] == 0 else (2,)))
    assert rep["factor_rows"] != 1 or rep["factor_pair"] == 0
    for k in ("trsv", "spmv", "setup"):
        assert 0 < rep[k + "_ms"] <= rep[k + "_default_ms"] * 1.0000001
    inf = S1.info()
    assert (inf["factor_rows"], inf["factor_pair"]) == (rep["factor_rows"], rep["factor_pair"])
    g = Grid(levels=levels)
    O = OracleSchwarz(g, P, gamma, curve="hilbert")
    r = uniform_pm1(71, g.N)
    tol = FP64_TOL if fdtype == "fp64" else FP32_TOL
    assert relerr(host(S1.apply(dvec(r))), O.apply(r)) <= tol
    S1.close()
    S2 = m.SFCSchwarz(**kw)
    inf2 = S2.info()
    assert (inf2["factor_rows"], inf2["factor_pair"]) == (rep["factor_rows"], rep["factor_pair"])
    assert (inf2["spmv_points"], inf2["spmv_window"]) == (rep["spmv_points"], rep["spmv_window"])
    rep2 = S2.tune("all", 2)
    assert rep2["tuned"] == 0 and rep2["setup_ms"] == rep["setup_ms"] and rep2["spmv_ms"] == rep["spmv_ms"]
    f0 = uniform_pm1(72, g.N)
    x, _ = S2.solve(dvec(f0), rtol=1e-12, method="fcg" if fdtype == "fp32" else "pcg")
    assert relerr(host(x), exact.solve(g, f0)) <= 1e-9
    S2.close()


def test_caller_workspace_sizes():
    """A caller's workspace of exactly the queried size works at any byte
    offset within its 256 bytes of slack; a buffer one byte short of the need
    at an aligned address fails with ENOMEM; a batch context accepts a
    workspace of its own query."""
    announce("caller workspace")
    kw = dict(levels=(5, 4), P=6, gamma=Fraction(1, 2), factor_dtype="fp64")
    nbytes = m.workspace_size(**kw)
    buf = torch.empty(nbytes + 512, dtype=torch.uint8, device=DEV)
    g = Grid(levels=(5, 4))
    f0 = uniform_pm1(2, g.N)
    ex = exact.solve(g, f0)
    base = buf.data_ptr()
    aligned = (-base) % 256
    for off in (aligned, aligned + 1, aligned + 255):
        S = m.SFCSchwarz(workspace=buf[off:off + nbytes], **kw)
        assert S.workspace_bytes == nbytes
        x, _ = S.solve(dvec(f0), rtol=1e-12)
        assert relerr(host(x), ex) <= 1e-9
        S.close()
    with pytest.raises(m.SfcddError) as e:
        m.SFCSchwarz(workspace=buf[aligned:aligned + nbytes - 257], **kw)
    assert e.value.status == m.ENOMEM
    with pytest.raises(ValueError):
        m.SFCSchwarz(workspace=torch.empty(nbytes, dtype=torch.float64, device=DEV), **kw)
    grids = [dict(levels=[5, 4], P=6), dict(levels=[3, 3], P=2)]
    B = m.SFCSchwarzBatch(grids, factor_dtype="fp64")
    want = B.workspace_bytes
    assert B.ws.numel() == want
    B.close()
    B = m.SFCSchwarzBatch(grids, factor_dtype="fp64", workspace=torch.empty(want, dtype=torch.uint8, device=DEV))
    assert B.workspace_bytes == want
    B.close()


def test_coarse_factor_precision_choice():
    """FP32 subdomain factors take an FP32 coarse factor only when the bound
    kappa(A) b_max / b_min on kappa(A_0) is at most 4096: the (7,6,5) grid
    with 256 subdomains (bound 3.0e3) does, the (14,1) grid with 128 (bound
    ~5e7) does not; FP64 factors never do."""
    announce("coarse precision choice")
    w = workloads()["c2"]
    for fdtype, want in (("fp32", 1), ("fp64", 0)):
        S = _solver(w.levels[0], w.P, w.gamma, factor_dtype=fdtype)
        assert S.info()["coarse_fp32"] == want, fdtype
        S.close()
    S = m.SFCSchwarz(levels=(14, 1), P=128, gamma=Fraction(1, 4), factor_dtype="fp32")
    assert S.info()["coarse_fp32"] == 0 and S.info()["coarse_inv_fp32"] == 1
    S.close()


@pytest.mark.parametrize("levels,P,gamma", [((6, 5, 5), 128, Fraction(1, 2)), ((7, 2), 11, Fraction(1, 2))])
def test_fp32_factors_with_fp64_coarse_operator(levels, P, gamma):
    """coarse_precision="fp64" keeps the coarse factor, inverse and solves in
    FP64 beside FP32 subdomain factors: the coarse-space identity of the
    balanced operator (C^{-1} A R_0^T c = R_0^T c) then holds to FP64
    rounding, and the application matches the oracle to the FP32 bar."""
    announce("fp64 coarse beside fp32 factors", levels, P, gamma)
    g = Grid(levels=levels)
    O = OracleSchwarz(g, P, gamma)
    S = _solver(levels, P, gamma, factor_dtype="fp32", coarse_precision="fp64", layout="sfc")
    inf = S.info()
    assert inf["coarse_fp32"] == 0 and inf["coarse_inv_fp32"] == 0
    r = uniform_pm1(41, g.N)
    sfc = S.partition()["sfc_index"]
    h = np.empty(g.N)
    h[sfc] = host(S.apply(dvec(r[sfc])))
    assert relerr(h, O.apply(r)) <= FP32_TOL
    cv = dvec(_coarse_vector(g.N, P, S.partition()["q"], 43))
    back = S.apply(S.matvec(cv))
    e = relerr(host(back), host(cv))
    print(f"coarse identity with the FP64 coarse operator: {e:.2e}", flush=True)
    assert e <= 1e-10
    S.close()


def test_largest_subdomain_single_piece_is_exact():
    """P = 1 at the largest subdomain the library takes (the (6, 7) grid:
    8001 points, 126 tiles): C^{-1} = A^{-1} exactly (the one subdomain is the
    whole grid), against the exact DST-I solve; PCG then converges in one
    iteration."""
    levels = (6, 7)
    announce("largest subdomain", levels)
    g = Grid(levels=levels)
    S = _solver(levels, 1, Fraction(1, 2), factor_dtype="fp64")
    assert S.info()["max_Ni"] == g.N == 8001
    r = uniform_pm1(41, g.N)
    assert relerr(host(S.apply(dvec(r))), exact.solve(g, r)) <= 1e-9
    x, info = S.solve(dvec(r), rtol=1e-8, method="pcg", plain_start=True, recursive=True)
    assert info["iterations"] <= 1
    assert relerr(host(x), exact.solve(g, r)) <= 1e-8
    S.close()


def test_concurrent_setups_on_two_streams():
    """Two host threads set up and solve on their own streams at the same
    time; their coarse setups share the device's internal stream (one after
    the other) and both solutions are right."""
    import threading
    announce("concurrent setups")
    cases = [((5, 4), 6, 51), ((4, 3, 3), 9, 52)]
    out = {}

    def work(levels, P, seed):
        g = Grid(levels=levels)
        f0 = uniform_pm1(seed, g.N)
        st = torch.cuda.Stream(device=DEV)
        with torch.cuda.stream(st):
            b = torch.tensor(f0, dtype=torch.float64, device=DEV)
            for _ in range(3):
                S = _solver(levels, P, Fraction(1, 2), factor_dtype="fp32")
                x, _ = S.solve(b, rtol=1e-12, method="fcg")
                S.close()
            st.synchronize()
            out[levels] = relerr(host(x), exact.solve(g, f0))

    ts = [threading.Thread(target=work, args=c) for c in cases]
    for t in ts:
        t.start()
    for t in ts:
        t.join(timeout=120)
    assert all(not t.is_alive() for t in ts)
    assert len(out) == 2 and all(e <= 1e-9 for e in out.values()), out
