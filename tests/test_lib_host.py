"""CPU tests of the C-ABI library: it loads, exports every declared entry
point, validates its parameters, and its host-side partition (eqs. sloc,
enlarge, omegai, q rule) equals the oracle's bit for bit."""
import os
import re
from fractions import Fraction

import numpy as np
import pytest

import paper_2110_11211_amd as m
from seeded_inputs import workloads
from oracle.grid import Grid
from oracle import partition as part
from oracle.schwarz import OracleSchwarz

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "sfcdd.h")


def test_library_exports_every_declared_symbol():
    names = re.findall(r"\b(sfcdd_[a-z_]+)\s*\(", open(HDR).read())
    names = sorted(set(names))
    assert len(names) >= 11
    L = m.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(m.EXPORTS) == set(names)


def _oracle_partition(levels, P, gamma, weighting="omega"):
    g = Grid(levels=levels)
    sets = part.overlap_sets(g.N, P, gamma)
    rng = [part.cyclic_range(S, g.N) for S in sets]
    mult = part.multiplicity(sets, g.N)
    om = part.omega(sets, mult) if weighting == "omega" else np.ones(P)
    return (np.array([r[0] for r in rng]), np.array([r[1] for r in rng]), om,
            part.coarse_rule_q(g.N, P))


@pytest.mark.parametrize("levels,P,gamma", [
    ((5, 5), 8, Fraction(1, 4)), ((7, 6, 5), 256, Fraction(1, 2)),
    ((3, 3, 3, 3, 3, 4), 512, Fraction(1, 4)), ((4, 3), 5, Fraction(3, 2)), ((3,), 7, Fraction(5, 2)),
    ((4, 4), 9, Fraction(2, 3)), ((2, 2, 2), 27, Fraction(0)), ((6, 2), 100, Fraction(7, 3)),
    ((5, 4, 3), 13, Fraction(1, 7)), ((3, 3), 2, Fraction(1, 2)), ((4,), 15, Fraction(1))])
def test_partition_host_matches_oracle(levels, P, gamma):
    ta, Ni, om, q = m.partition_host(levels=levels, P=P, gamma=gamma)
    ota, oNi, oom, oq = _oracle_partition(levels, P, gamma)
    assert np.array_equal(ta, ota) and np.array_equal(Ni, oNi)
    assert np.array_equal(om, oom) and q == oq


def test_partition_host_random_small_cases():
    """Random small grids, P and gamma (including P = N, gamma beyond full
    overlap, and wrapping subdomains) against the oracle's set construction."""
    rng = np.random.default_rng(2024)
    for _ in range(60):
        d = int(rng.integers(1, 3))
        levels = tuple(int(v) for v in rng.integers(1, 5, size=d))
        N = Grid(levels=levels).N
        P = int(rng.integers(1, N + 1))
        gamma = Fraction(int(rng.integers(0, 13)), int(rng.integers(1, 5)))
        ta, Ni, om, q = m.partition_host(levels=levels, P=P, gamma=gamma)
        ota, oNi, oom, oq = _oracle_partition(levels, P, gamma)
        case = (levels, P, gamma)
        assert np.array_equal(ta, ota) and np.array_equal(Ni, oNi), case
        assert np.array_equal(om, oom) and q == oq, case


def test_partition_host_ct_layer():
    w = workloads()["c4"]
    for lv in w.levels[::7]:
        ta, Ni, om, q = m.partition_host(levels=lv, P=w.P, gamma=w.gamma)
        ota, oNi, oom, oq = _oracle_partition(lv, w.P, w.gamma)
        assert np.array_equal(ta, ota) and np.array_equal(Ni, oNi)
        assert np.array_equal(om, oom) and q == oq


@pytest.mark.slow
def test_partition_host_large_grid():
    w = workloads()["c5"]
    ta, Ni, om, q = m.partition_host(levels=w.levels[0], P=w.P, gamma=w.gamma)
    ota, oNi, oom, oq = _oracle_partition(w.levels[0], w.P, w.gamma)
    assert np.array_equal(ta, ota) and np.array_equal(Ni, oNi)
    assert np.array_equal(om, oom) and q == oq == 4
    assert Ni.min() == 2520 and Ni.max() == 2522


def test_partition_host_weighting_none_and_explicit_q():
    ta, Ni, om, q = m.partition_host(levels=(5, 5), P=8, gamma=Fraction(1, 2), weighting="none", q=3)
    assert np.all(om == 1.0) and q == 3


def test_partition_host_1d_npts():
    ta, Ni, om, q = m.partition_host(npts=[256 * 16], P=16, gamma=Fraction(1, 2), q=16)
    S = OracleSchwarz(Grid(npts=[256 * 16]), 16, Fraction(1, 2), q=16, factor=False)
    assert np.array_equal(ta, S.ta) and np.array_equal(Ni, S.Ni) and np.allclose(om, 0.5)


@pytest.mark.parametrize("kw,code", [
    (dict(levels=(3, 3), P=0), m.EINVAL), (dict(levels=(3, 3), P=50), m.EINVAL),
    (dict(levels=(3, 3), P=4, gamma=Fraction(-1, 2)), m.EINVAL),
    (dict(levels=(3, 3), P=4, q=20), m.EINVAL), (dict(levels=(11,) * 6, P=4), m.EOVERFLOW),
    (dict(levels=(16, 16), P=4), m.EOVERFLOW), (dict(levels=(0, 3), P=4), m.EINVAL),
    (dict(levels=(3, 3), P=4, coeff=(1.0, -1.0)), m.EINVAL),
    (dict(npts=[8193], P=1), m.EINVAL),                          # a subdomain above 8192 points
    (dict(npts=[1 << 18], P=2048, q=128), m.EINVAL)])            # coarse size qP above 131072
def test_invalid_parameters(kw, code):
    with pytest.raises(m.SfcddError) as e:
        m.workspace_size(**kw)
    assert e.value.status == code


def test_size_limits_accepted_at_the_bound():
    assert m.workspace_size(npts=[8192], P=1) > 8192 * 8192 * 4
    assert m.workspace_size(npts=[1 << 18], P=2048, q=64) > 0   # qP = 131072


def test_noalloc_setup_rejects_oversize_before_any_device_work():
    """The allocation-free setup checks the planned workspace against its
    static array on the host, before any HIP call: ENOMEM with the sizes."""
    import ctypes
    prm, keep = m.make_params(levels=(7, 6, 5), P=256, gamma=Fraction(1, 2), factor_dtype="fp32")
    ctx = ctypes.c_void_p()
    st = m.lib().sfcdd_setup_noalloc(ctypes.byref(prm), None, ctypes.byref(ctx))
    assert st == m.ENOMEM and not ctx.value
    msg = m.lib().sfcdd_last_error(None).decode()
    assert str(m.NOALLOC_WORKSPACE_BYTES) in msg and "allocation-free" in msg


def test_iterative_coarse_rule_and_validation():
    """The iterative coarse solver keeps the four-levels-coarser rule uncapped
    (q = 64 on the 8.26 M-unknown grid with 4096 subdomains, where the dense
    solver caps it at 4), allows coarse sizes up to 2^22, validates its
    tolerance, and is refused for batches."""
    import ctypes
    kw = dict(levels=(8, 8, 7), P=4096, gamma=Fraction(1, 8))
    assert m.partition_host(**kw)[3] == 4
    assert m.partition_host(coarse_solver="iterative", **kw)[3] == 64
    assert m.partition_host(levels=(10, 10), P=1024, gamma=Fraction(1, 4), coarse_solver="iterative")[3] == 32
    with pytest.raises(m.SfcddError) as e:
        m.workspace_size(coarse_solver="iterative", coarse_tol=1.5, **kw)
    assert e.value.status == m.EINVAL
    with pytest.raises(m.SfcddError) as e:        # dense coarse size limit
        m.workspace_size(levels=(8, 8, 7), P=4096, gamma=Fraction(1, 8), q=64)
    assert e.value.status == m.EINVAL
    arr = (m.Params * 2)()
    keep = []
    for k in range(2):
        prm, kp = m.make_params(levels=(5, 5), P=8, gamma=Fraction(1, 4), coarse_solver="iterative")
        arr[k] = prm
        keep.append(kp)
    n = ctypes.c_size_t()
    assert m.lib().sfcdd_workspace_size_batch(2, arr, ctypes.byref(n)) == m.EINVAL


def test_workspace_grows_with_factor_precision():
    a = m.workspace_size(levels=(7, 6, 5), P=256, gamma=Fraction(1, 2), factor_dtype="fp32")
    b = m.workspace_size(levels=(7, 6, 5), P=256, gamma=Fraction(1, 2), factor_dtype="fp64")
    assert b > a > 1.9e9


def test_ct_layout_against_oracle():
    """Grids, layers, weights and subdomain counts of the combination-technique
    binding (host logic) against the oracle's enumeration (eq. combi, eq.
    Pchoice), and the capped P never exceeds a grid's size."""
    from paper_2110_11211_amd.ct import ct_layout
    from oracle import ct as oct
    from oracle.grid import Grid
    for d in range(1, 6):
        for L in range(d, d + 5):
            for phat in (1, 4):
                got = ct_layout(d, L, phat)
                ref = oct.ct_grids(d, L)
                assert [(lv, i, w) for lv, i, w, _ in got] == ref
                for lv, i, _, P in got:
                    N = Grid(levels=lv).N
                    assert P == min(oct.subdomains_per_grid(d, i, phat), N)
