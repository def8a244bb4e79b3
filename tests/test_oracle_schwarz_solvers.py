"""Pins of the oracle's preconditioners, solvers and gradient."""
import os
from fractions import Fraction

import numpy as np
import pytest

from seeded_inputs import uniform_pm1, workloads
from oracle.grid import Grid
from oracle.schwarz import OracleSchwarz
from oracle import exact, solvers, grad
from oracle import partition as part

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _paper_pins():
    out = {}
    for l in open(os.path.join(GOLD, "paper_d1_iterations.txt")):
        if l.strip() and not l.startswith("#"):
            k, v = l.split()[:2]
            out[k] = float(v)
    return out


SMALL = [((3, 3), 4, Fraction(1, 2), 2), ((2, 3, 2), 5, Fraction(1, 4), 3), ((4, 3), 6, Fraction(3, 4), 2),
         ((5,), 3, Fraction(1, 1), 4)]


@pytest.mark.parametrize("levels,P,gamma,q", SMALL)
def test_local_matrices_are_principal_submatrices_and_spd(levels, P, gamma, q):
    g = Grid(levels=levels)
    S = OracleSchwarz(g, P, gamma, q=q, factor=False)
    A = g.matrix().toarray()
    for i in range(P):
        nat = S.sfc_index[S.orders[i]]
        Ai = S.local_matrix(i)
        assert np.array_equal(Ai, A[np.ix_(nat, nat)])
        assert np.linalg.eigvalsh(Ai).min() > 0


@pytest.mark.parametrize("levels,P,gamma,q", SMALL)
def test_coarse_matrix_brute_force(levels, P, gamma, q):
    """(A_0)_{IJ} = sum over p in block I, p' in block J of A_{pp'} (eq. csm),
    summed directly over stencil pairs."""
    g = Grid(levels=levels, coeff=[1.0 + 0.5 * j for j in range(len(levels))])
    S = OracleSchwarz(g, P, gamma, q=q, factor=False)
    blocks = part.coarse_blocks(g.N, P, q)
    blk = np.empty(g.N, dtype=int)
    for I, (s, sz) in enumerate(blocks):
        blk[s:s + sz] = I
    K = g.coords()
    A0 = np.zeros((q * P, q * P))
    for nat in range(g.N):
        I = blk[S.pos[nat]]
        A0[I, I] += sum(2 * g.c[j] for j in range(g.d))
        for j in range(g.d):
            for s in (-1, 1):
                kk = K[nat, j] + s
                if 1 <= kk <= g.n[j]:
                    A0[I, blk[S.pos[nat + s * g.stride[j]]]] -= g.c[j]
    assert np.allclose(S.A0, A0, rtol=1e-14, atol=0)


@pytest.mark.parametrize("variant", ["additive", "balanced"])
@pytest.mark.parametrize("levels,P,gamma,q", SMALL)
def test_preconditioner_symmetric_positive(variant, levels, P, gamma, q):
    g = Grid(levels=levels)
    S = OracleSchwarz(g, P, gamma, q=q, variant=variant)
    C = S.dense_preconditioner()
    assert np.allclose(C, C.T, atol=1e-12 * np.abs(C).max())
    assert np.linalg.eigvalsh(0.5 * (C + C.T)).min() > 0


def test_D_weighting_symmetric_only_for_half_integer_gamma():
    g = Grid(levels=(3, 3))
    C = OracleSchwarz(g, 4, Fraction(1, 2), q=2, weighting="D", variant="additive").dense_preconditioner()
    assert np.allclose(C, C.T, atol=1e-12 * np.abs(C).max())
    C = OracleSchwarz(g, 4, Fraction(1, 3), q=2, weighting="D", variant="additive").dense_preconditioner()
    assert not np.allclose(C, C.T, atol=1e-6 * np.abs(C).max())


@pytest.mark.parametrize("levels,P,gamma,q", SMALL)
def test_balanced_is_identity_on_coarse_space(levels, P, gamma, q):
    """With G = I - AF: C_bal^{-1} A v = v for every v = R_0^T c."""
    g = Grid(levels=levels)
    S = OracleSchwarz(g, P, gamma, q=q, variant="balanced")
    c = uniform_pm1(5, q * P)
    v_s = S.R0.T @ c
    v = S.from_s(v_s)
    assert np.allclose(S.apply(S.matvec(v)), v, atol=1e-11 * np.abs(v).max())


@pytest.mark.parametrize("levels,P,gamma,q", SMALL)
def test_balancing_start_keeps_residuals_in_kernel_of_R0(levels, P, gamma, q):
    """From x_0 = F b the residual has R_0 r = 0, CG keeps it there, and on
    such r the balanced operator equals (I - F A) C1^{-1} r (t = F r vanishes)."""
    g = Grid(levels=levels)
    S = OracleSchwarz(g, P, gamma, q=q, variant="balanced")
    b = uniform_pm1(6, g.N)
    nb = np.linalg.norm(S.R0 @ S.to_s(b))
    x0 = S.balancing_start(b)
    r0 = S.to_s(b - S.matvec(x0))
    assert np.linalg.norm(S.R0 @ r0) <= 1e-12 * nb
    x3, _, _ = solvers.pcg(S.A_nat, b, S.apply, x0=x0, rtol=1e-300, maxit=3)
    r3 = S.to_s(b - S.matvec(x3))
    assert np.linalg.norm(S.R0 @ r3) <= 1e-11 * nb
    v = S.to_s(uniform_pm1(7, g.N))
    r = v - S.A @ S.coarse_s(v)                      # R_0 r = 0
    y = S.fine_s(r)
    proj = y - S.coarse_s(S.A @ y)
    assert np.allclose(S.apply_s(r), proj, atol=1e-12 * np.abs(proj).max())


@pytest.mark.parametrize("levels,P,gamma,q", SMALL)
def test_two_level_forms_reproduce_the_coarse_residual(levels, P, gamma, q):
    """R_0 A C^{-1} r = R_0 r for the balanced and the deflated forms
    (R_0 A G^T = 0 and R_0 A F = R_0), not for the additive one; on r with
    R_0 r = 0 the balanced and deflated forms coincide."""
    g = Grid(levels=levels)
    r = uniform_pm1(8, g.N)
    ops = {v: OracleSchwarz(g, P, gamma, q=q, variant=v) for v in ("balanced", "deflated", "additive")}
    for v in ("balanced", "deflated"):
        S = ops[v]
        lhs = S.R0 @ (S.A @ S.apply_s(S.to_s(r)))
        assert np.allclose(lhs, S.R0 @ S.to_s(r), atol=1e-10 * np.abs(S.R0 @ S.to_s(r)).max())
    Sa = ops["additive"]
    lhs = Sa.R0 @ (Sa.A @ Sa.apply_s(Sa.to_s(r)))
    assert not np.allclose(lhs, Sa.R0 @ Sa.to_s(r), atol=1e-6 * np.abs(Sa.R0 @ Sa.to_s(r)).max())
    Sb, Sd = ops["balanced"], ops["deflated"]
    v = Sb.to_s(uniform_pm1(9, g.N))
    r0 = v - Sb.A @ Sb.coarse_s(v)                     # R_0 r0 = 0
    assert np.allclose(Sb.apply_s(r0), Sd.apply_s(r0), atol=1e-12 * np.abs(Sb.apply_s(r0)).max())


def test_single_subdomain_is_exact():
    """P = 1: the only subdomain is the whole grid, so C_bal^{-1} = A^{-1}
    (PCG converges in one step) and additive PCG needs at most two."""
    g = Grid(levels=(3, 4))
    f = uniform_pm1(1, g.N)
    xs = exact.solve(g, f)
    S = OracleSchwarz(g, 1, Fraction(1, 2), q=4, variant="balanced")
    assert np.allclose(S.apply(f), xs, rtol=0, atol=1e-12 * np.abs(xs).max())
    x, it, _ = solvers.pcg(S.A_nat, f, S.apply, rtol=1e-12)
    assert it == 1
    S = OracleSchwarz(g, 1, Fraction(1, 2), q=4, variant="additive")
    x, it, _ = solvers.pcg(S.A_nat, f, S.apply, rtol=1e-12)
    assert it <= 2


def test_full_overlap_one_level_is_exact():
    """gamma >= (P-1)/2: every subdomain is the whole grid, every point has
    multiplicity P, omega_i = 1/P, so the weighted one-level operator is A^{-1}."""
    g = Grid(levels=(3, 3))
    f = uniform_pm1(2, g.N)
    S = OracleSchwarz(g, 5, Fraction(2), q=2, variant="onelevel")
    assert np.all(S.Ni == g.N) and np.allclose(S.omega, 0.2)
    assert np.allclose(S.apply(f), exact.solve(g, f), atol=1e-12)


def test_pcg_c1_matches_exact_solution():
    w = workloads()["c1"]
    g = Grid(levels=w.levels[0])
    S = OracleSchwarz(g, w.P, w.gamma)
    f = w.rhs()
    x, it, _ = solvers.pcg(S.A_nat, f, S.apply, rtol=1e-12)
    xs = exact.solve(g, f)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    assert 10 <= it <= 60


def test_iterations_independent_of_P_for_fixed_N_over_P():
    """Weak scaling (Sec. 4.1): balanced omega-PCG counts level off as P grows."""
    its = []
    for P in (64, 128):
        g = Grid(npts=[256 * P])
        S = OracleSchwarz(g, P, Fraction(1, 2), q=16)
        x0 = solvers.paper_start(S.A_nat, 11, g.N)
        its.append(solvers.pcg(S.A_nat, np.zeros(g.N), S.apply, x0=x0, energy_tol=1e-8)[1])
    assert abs(its[0] - its[1]) <= 1
    assert max(its) <= _paper_pins()["pcg_balanced_omega_max"]


def test_lanczos_matches_dense_spectrum():
    g = Grid(levels=(4, 3))
    S = OracleSchwarz(g, 6, Fraction(1, 2), q=2)
    lmin, lmax = solvers.dense_spectrum(S.A_nat.toarray(), S.dense_preconditioner())
    a, b = solvers.cg_coefficients(S.A_nat, uniform_pm1(4, g.N), S.apply, 60)
    emin, emax = solvers.lanczos_extremes(a, b)
    assert abs(emin - lmin) <= 1e-6 * lmin and abs(emax - lmax) <= 1e-6 * lmax


def test_richardson_contracts_at_optimal_rate():
    """eq. (redrate): with xi* the energy norm of the error contracts by at
    most rho* = 1 - 2/(1+kappa) per step, and no more slowly asymptotically."""
    g = Grid(levels=(4, 4))
    S = OracleSchwarz(g, 6, Fraction(1, 2), q=2)
    A = S.A_nat
    lmin, lmax = solvers.dense_spectrum(A.toarray(), S.dense_preconditioner())
    xi, rho = solvers.optimal_damping(lmin, lmax)
    assert abs(rho - (lmax - lmin) / (lmax + lmin)) < 1e-14
    x = solvers.paper_start(A, 3, g.N)
    en = [1.0]
    for _ in range(40):
        x = x + xi * S.apply(-(A @ x))
        en.append(np.sqrt(float(x @ (A @ x))))
    ratios = np.array(en[1:]) / np.array(en[:-1])
    assert np.all(ratios <= rho * (1 + 1e-9))
    assert ratios[-10:].mean() >= 0.7 * rho


def _d1_counts(P, variant, weighting):
    g = Grid(npts=[256 * P])
    S = OracleSchwarz(g, P, Fraction(1, 2), q=16, weighting=weighting, variant=variant)
    A = S.A_nat
    x0 = solvers.paper_start(A, 11, g.N)
    b = np.zeros(g.N)
    it_cg = solvers.pcg(A, b, S.apply, x0=x0, energy_tol=1e-8)[1]
    a, bb = solvers.cg_coefficients(A, uniform_pm1(99, g.N), S.apply, 150)
    xi, _ = solvers.optimal_damping(*solvers.lanczos_extremes(a, bb))
    it_r = solvers.richardson(A, b, S.apply, xi, x0=x0, energy_tol=1e-8)[1]
    return it_r, it_cg


@pytest.mark.slow
def test_paper_d1_balanced_vs_additive():
    """Sec. 4.1 (d = 1, S = 8, q = 16, gamma = 1/2): balanced Richardson needs
    about 7x (unweighted) / 6x (omega) fewer iterations than additive,
    balanced PCG nearly half; the three balanced weightings coincide."""
    pins = _paper_pins()
    P = 32
    ra_n, ca_n = _d1_counts(P, "additive", "none")
    ra_w, ca_w = _d1_counts(P, "additive", "omega")
    rb_n, cb_n = _d1_counts(P, "balanced", "none")
    rb_w, cb_w = _d1_counts(P, "balanced", "omega")
    rb_d, cb_d = _d1_counts(P, "balanced", "D")
    assert rb_n == rb_w == rb_d and abs(cb_n - cb_w) <= 1 and cb_w == cb_d
    assert ra_w < ra_n                                   # omega weighting helps additive Richardson
    assert 0.7 * pins["ratio_richardson_unweighted"] <= ra_n / rb_n <= 1.3 * pins["ratio_richardson_unweighted"]
    assert 0.7 * pins["ratio_richardson_weighted"] <= ra_w / rb_w <= 1.3 * pins["ratio_richardson_weighted"]
    assert 0.35 <= cb_w / ca_w <= 0.7
    assert rb_w <= pins["richardson_balanced_omega_limit"]
    assert cb_w <= pins["pcg_balanced_omega_max"]


@pytest.mark.parametrize("levels,coeff", [((3, 4), (0.5, 2.0)), ((2, 3, 2), (0.2, 1.0, 5.0))])
def test_adjoint_gradient_matches_finite_differences(levels, coeff):
    g = Grid(levels=levels, coeff=coeff)
    f = uniform_pm1(8, g.N)
    u = exact.solve(g, f)
    gf, ga = grad.adjoint_gradient(g, u, u)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(g.N)
    eps = 1e-4
    fd = (grad.objective(g, f + eps * v) - grad.objective(g, f - eps * v)) / (2 * eps)
    assert abs(fd - gf @ v) <= 1e-7 * abs(fd)
    for j in range(g.d):
        a_p = list(coeff); a_m = list(coeff)
        h = 1e-5 * coeff[j]
        a_p[j] += h; a_m[j] -= h
        fd = (grad.objective(Grid(levels=levels, coeff=a_p), f)
              - grad.objective(Grid(levels=levels, coeff=a_m), f)) / (2 * h)
        assert abs(fd - ga[j]) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("levels,P,gamma,q", [((5, 4), 6, Fraction(1, 2), 0), ((4, 3, 3), 9, Fraction(1, 4), 2),
                                              ((7,), 5, Fraction(1, 3), 3), ((3, 5), 7, Fraction(1), 0)])
def test_coarse_matrix_is_m_matrix_within_condition_bound(levels, P, gamma, q):
    """The facts the FP32 coarse path rests on: A_0 = R_0 A R_0^T is an
    M-matrix (non-positive off-diagonal entries), so L_0^{-1} is entrywise
    non-negative; and kappa(A_0) <= kappa(A) b_max / b_min (Rayleigh quotients
    with R_0 R_0^T = diag(block sizes)), kappa(A) from the stencil's extreme
    sine eigenvalues."""
    g = Grid(levels=levels)
    S = OracleSchwarz(g, P, gamma, q=q or None, factor=False)
    A0 = S.A0
    off = A0 - np.diag(np.diag(A0))
    assert off.max() <= 0.0
    L0 = np.linalg.cholesky(A0)
    X0 = np.linalg.inv(L0)
    assert X0.min() >= -1e-12 * np.abs(X0).max()
    ev = np.linalg.eigvalsh(A0)
    lam = np.linalg.eigvalsh(g.matrix().toarray())
    bsz = np.asarray(S.R0.sum(axis=1)).ravel()
    assert bsz.min() >= 1
    assert ev[-1] / ev[0] <= (lam[-1] / lam[0]) * bsz.max() / bsz.min() * (1 + 1e-12)


def _recorded_cg(A, b, M, flexible, x0=None, rtol=1e-12, maxit=400):
    """Runs the oracle's PCG with M wrapped so that every (r, z) pair it
    applies is kept; the search directions are rebuilt from the z's and the
    returned beta's (p_0 = z_0, p_k = z_k + beta_{k-1} p_{k-1})."""
    seen = []

    def Mrec(r):
        z = M(r)
        seen.append((r.copy(), z.copy()))
        return z

    x, it, info = solvers.pcg(A, b, Mrec, x0=x0, rtol=rtol, maxit=maxit, flexible=flexible)
    ps = [seen[0][1]]
    for k, beta in enumerate(info["betas"]):
        ps.append(seen[k + 1][1] + beta * ps[-1])
    return x, it, seen, ps


def _local_a_orthogonality(A, seen, ps):
    """Largest |p_{k+1}^T A p_k| / (||p_{k+1}||_A ||p_k||_A) and largest
    |p_k^T r_{k+1}| / (||p_k|| ||r_{k+1}||) over the run."""
    worst_ap, worst_pr = 0.0, 0.0
    for k in range(len(ps) - 1):
        Ap = A @ ps[k]
        nk = np.sqrt(float(ps[k] @ Ap))
        nk1 = np.sqrt(float(ps[k + 1] @ (A @ ps[k + 1])))
        worst_ap = max(worst_ap, abs(float(ps[k + 1] @ Ap)) / (nk * nk1))
        r1 = seen[k + 1][0]
        worst_pr = max(worst_pr, abs(float(ps[k] @ r1)) / (np.linalg.norm(ps[k]) * np.linalg.norm(r1)))
    return worst_ap, worst_pr


def test_flexible_cg_keeps_consecutive_directions_a_orthogonal():
    """Flexible CG (Sec. 3.3, the remedy for a non-symmetric preconditioner):
    with beta = z_{k+1}^T (r_{k+1} - r_k) / z_k^T r_k every new direction is
    A-orthogonal to the previous one and every residual is orthogonal to the
    last direction, for any preconditioner.  With the D_i weights at
    gamma = 1/4 (non-symmetric) the flexible branch keeps both to rounding,
    the standard beta does not, and the flexible iteration reaches the exact
    DST-I solution."""
    levels, P, gamma = (5, 4, 3), 12, Fraction(1, 4)
    g = Grid(levels=levels)
    S = OracleSchwarz(g, P, gamma, weighting="D", variant="balanced")
    f = uniform_pm1(10, g.N)
    xs = exact.solve(g, f)
    x, it, seen, ps = _recorded_cg(S.A_nat, f, S.apply, flexible=True)
    ap, pr = _local_a_orthogonality(S.A_nat, seen, ps)
    assert ap <= 1e-9 and pr <= 1e-9, (ap, pr)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
    _, _, seen_s, ps_s = _recorded_cg(S.A_nat, f, S.apply, flexible=False, maxit=15)
    ap_s, _ = _local_a_orthogonality(S.A_nat, seen_s, ps_s)
    assert ap_s >= 1e-6, ap_s


def test_flexible_cg_equals_pcg_for_a_symmetric_preconditioner():
    """With a fixed symmetric positive definite preconditioner z_{k+1}^T r_k = 0,
    so the flexible beta equals the standard one: same iteration count and the
    same iterate (the d = 2 workload, balanced omega-weighted form, and a d = 3
    grid from the balancing start)."""
    w = workloads()["c1"]
    g = Grid(levels=w.levels[0])
    S = OracleSchwarz(g, w.P, w.gamma)
    f = w.rhs()
    x_p, it_p, _ = solvers.pcg(S.A_nat, f, S.apply, rtol=1e-10)
    x_f, it_f, _ = solvers.pcg(S.A_nat, f, S.apply, rtol=1e-10, flexible=True)
    assert it_p == it_f
    assert np.linalg.norm(x_p - x_f) <= 1e-10 * np.linalg.norm(x_p)
    g3 = Grid(levels=(4, 3, 3))
    S3 = OracleSchwarz(g3, 10, Fraction(1, 2))
    f3 = uniform_pm1(4, g3.N)
    x0 = S3.balancing_start(f3)
    x_p, it_p, _ = solvers.pcg(S3.A_nat, f3, S3.apply, x0=x0, rtol=1e-10)
    x_f, it_f, _ = solvers.pcg(S3.A_nat, f3, S3.apply, x0=x0, rtol=1e-10, flexible=True)
    assert it_p == it_f
    assert np.linalg.norm(x_p - x_f) <= 1e-10 * np.linalg.norm(x_p)
