"""GPU test of the allocation-free setup (sfcdd_setup_noalloc): the library's
static per-device workspace in place of a caller buffer.  Two setups in a
row, the second on a smaller grid, each checked against the same setup on a
caller-owned workspace (sfcdd_setup) through the C ABI: the same kernels on
the same inputs, so the preconditioner applications, the matrix-vector
products and the solves agree bit for bit.  The first context is stale once
the second setup has taken the array over."""
from fractions import Fraction

import numpy as np
import pytest
import torch

import paper_2110_11211_amd as m
from seeded_inputs import uniform_pm1
from gpu_common import DEV, announce, dvec, host, relerr

pytestmark = pytest.mark.gpu

CASES = [
    # (levels, P, gamma, factor dtype, curve, method): the second is smaller
    ((5, 5, 4), 16, Fraction(1, 2), "fp32", "hilbert", "fcg"),
    ((5, 5), 8, Fraction(1, 4), "fp64", "zorder", "pcg"),
]


def _kw(levels, P, gamma, fdtype, curve):
    return dict(levels=levels, P=P, gamma=gamma, factor_dtype=fdtype, curve=curve)


def test_noalloc_setup_matches_workspace_setup_twice():
    prev = None
    sizes = []
    for k, (levels, P, gamma, fdtype, curve, method) in enumerate(CASES):
        kw = _kw(levels, P, gamma, fdtype, curve)
        announce("noalloc", k, levels, P, gamma, fdtype, curve)
        nbytes = m.workspace_size(**kw)
        assert nbytes <= m.NOALLOC_WORKSPACE_BYTES
        sizes.append(nbytes)
        ref = m.SFCSchwarz(device=DEV, **kw)
        sta = m.SFCSchwarz(device=DEV, workspace="static", **kw)
        assert sta.ws is None
        N = ref.N
        g = dvec(uniform_pm1(100 + k, N))
        h_ref = host(ref.apply(g))
        h_sta = host(sta.apply(g))
        assert np.array_equal(h_ref, h_sta), f"apply differs: {relerr(h_sta, h_ref):.3e}"
        y_ref = host(ref.matvec(g))
        y_sta = host(sta.matvec(g))
        assert np.array_equal(y_ref, y_sta)
        b = dvec(uniform_pm1(200 + k, N))
        x_ref, i_ref = ref.solve(b, rtol=1e-10, method=method)
        x_sta, i_sta = sta.solve(b, rtol=1e-10, method=method)
        assert i_ref["iterations"] == i_sta["iterations"]
        assert np.array_equal(host(x_ref), host(x_sta))
        # the solution also satisfies A x = b to the requested residual
        r = host(b) - host(sta.matvec(x_sta))
        assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(host(b))
        print(f"noalloc case {k}: N={N} workspace {nbytes} B, apply/matvec/solve bit-identical, "
              f"{i_sta['iterations']} iterations", flush=True)
        if prev is not None:
            # the earlier allocation-free context lost its workspace to this setup
            with pytest.raises(m.SfcddError) as e:
                prev.apply(dvec(np.zeros(prev.N)))
            assert e.value.status == m.EINVAL
            prev.close()
        ref.close()
        prev = sta
    prev.close()
    assert sizes[1] < sizes[0]
    torch.cuda.synchronize()


def test_noalloc_rejects_a_problem_larger_than_the_static_workspace():
    kw = _kw((7, 6, 5), 256, Fraction(1, 2), "fp32", "hilbert")
    assert m.workspace_size(**kw) > m.NOALLOC_WORKSPACE_BYTES
    with pytest.raises(m.SfcddError) as e:
        m.SFCSchwarz(device=DEV, workspace="static", **kw)
    assert e.value.status == m.ENOMEM
    assert "allocation-free" in str(e.value)
