"""Pins of the oracle's curve order and partition (bit-exact index work)."""
import functools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle.grid import Grid
from oracle.sfc import sfc_order, morton_keys, hilbert_keys, hilbert_transpose
from oracle import partition as part

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_zorder_golden_3x3():
    rows = [list(map(int, l.split())) for l in open(os.path.join(GOLD, "zorder_l2x2.txt"))
            if l.strip() and not l.startswith("#")]
    g = Grid(levels=(2, 2))
    sfc_index, pos = sfc_order(g)
    keys = morton_keys(g)
    assert list(sfc_index) == [r[3] for r in rows]
    assert [int(keys[r[3]]) for r in rows] == [r[2] for r in rows]


def _less_msb(a, b):
    """True if the highest set bit of a is below that of b (a < b and a < a^b)."""
    return a < b and a < (a ^ b)


def _zcmp(p, q):
    """Z-order comparison of two coordinate tuples without building keys: the
    dimension whose coordinates differ in the most significant bit decides;
    on a tie in bit level the higher dimension wins (it sits higher in the key)."""
    msd = len(p) - 1
    for dim in range(len(p) - 2, -1, -1):
        if _less_msb(p[msd] ^ q[msd], p[dim] ^ q[dim]):
            msd = dim
    return (p[msd] > q[msd]) - (p[msd] < q[msd])


@pytest.mark.parametrize("levels", [(3, 3), (4, 2), (2, 3, 4), (3, 1, 2, 2), (1, 5)])
def test_zorder_matches_comparator_sort(levels):
    """Key interleave + argsort agrees with a comparator sort on scaled coordinates."""
    g = Grid(levels=levels)
    nres = max(levels)
    K = g.coords()
    pts = [tuple(int(K[i, j]) << (nres - levels[j]) for j in range(g.d)) for i in range(g.N)]
    order = sorted(range(g.N), key=functools.cmp_to_key(lambda a, b: _zcmp(pts[a], pts[b])))
    sfc_index, pos = sfc_order(g)
    assert list(sfc_index) == order
    assert np.array_equal(pos[sfc_index], np.arange(g.N))


def test_zorder_1d_and_reduced_is_identity():
    for g in [Grid(npts=[1000]), Grid(levels=(7,)), Grid(levels=(6, 1, 1, 1))]:
        sfc_index, _ = sfc_order(g)
        assert np.array_equal(sfc_index, np.arange(g.N))


def test_key_width_limit():
    with pytest.raises(OverflowError):
        sfc_order(Grid(levels=(11,) * 6))   # 66 key bits


CASES = [(961, 8, Fraction(1, 4)), (100, 7, Fraction(1, 2)), (101, 7, Fraction(3, 2)),
         (50, 3, Fraction(1, 1)), (17, 5, Fraction(2, 5)), (64, 4, Fraction(5, 2)),
         (30, 2, Fraction(1, 2)), (9, 9, Fraction(1, 3)), (1000, 13, Fraction(7, 8)),
         (23, 4, Fraction(0)), (40, 1, Fraction(1, 2))]


@pytest.mark.parametrize("N,P,gamma", CASES)
def test_overlap_closed_form(N, P, gamma):
    """(ta_i, N_i) from the set union of eq. (enlarge) against the closed form
    len = sum_{|k|<=F} ~N_{i+k} + ceil(eta ~N_{i-F-1}) + floor(eta ~N_{i+F+1})."""
    sizes = part.piece_sizes(N, P)
    starts = part.piece_starts(N, P)
    assert sizes.sum() == N and sizes.max() - sizes.min() <= 1
    assert list(sizes) == sorted(sizes, reverse=True)
    F = math.floor(gamma)
    eta = gamma - F
    for i, S in enumerate(part.overlap_sets(N, P, gamma)):
        ta, Ni, order = part.cyclic_range(S, N)
        nl = math.ceil(eta * int(sizes[(i - F - 1) % P]))
        nr = math.floor(eta * int(sizes[(i + F + 1) % P]))
        ln = sum(int(sizes[(i + k) % P]) for k in range(-F, F + 1)) + nl + nr
        if ln >= N:
            assert (ta, Ni) == (0, N)
        else:
            assert Ni == ln
            assert ta == (int(starts[(i - F) % P]) - nl) % N
        assert set(order.tolist()) == set(S.tolist())


@pytest.mark.parametrize("N,P", [(97, 7), (256, 8), (1000, 12), (33, 5), (64, 16)])
@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_lemma_uniform_multiplicity(N, P, n):
    """Lemma (Sec. 3.4): gamma = n/2, n <= P-1 gives multiplicity 2 gamma + 1
    at every point and omega_i = 1/(2 gamma + 1)."""
    if n > P - 1:
        pytest.skip("lemma needs n <= P-1")
    sets = part.overlap_sets(N, P, Fraction(n, 2))
    m = part.multiplicity(sets, N)
    assert np.all(m == n + 1)
    assert np.allclose(part.omega(sets, m), 1.0 / (n + 1))


@pytest.mark.parametrize("N,P,gamma", CASES)
def test_partition_of_unity(N, P, gamma):
    """eq. (pum) with D_i from eq. (Di): sum_i R_i^T D_i R_i = I."""
    sets = part.overlap_sets(N, P, gamma)
    m = part.multiplicity(sets, N)
    acc = np.zeros(N)
    for S, w in zip(sets, part.point_weights(sets, m)):
        acc[S] += w
    assert np.allclose(acc, 1.0)
    om = part.omega(sets, m)
    assert np.all(om <= 1.0) and np.all(om > 0)


def test_omega_is_one_when_a_point_is_uncovered_by_others():
    """gamma < 1/2 leaves points owned by one subdomain, so omega_i = 1."""
    sets = part.overlap_sets(961, 8, Fraction(1, 4))
    m = part.multiplicity(sets, 961)
    assert np.all(part.omega(sets, m) == 1.0)


@pytest.mark.parametrize("N,P,q", [(961, 8, 4), (248031, 256, 32), (100, 7, 3), (50, 5, 10)])
def test_coarse_blocks(N, P, q):
    """eq. (restr): blocks tile every piece, sizes differ by at most one with
    the larger ones first, and R_0 has exactly one 1 per column."""
    blocks = part.coarse_blocks(N, P, q)
    starts = part.piece_starts(N, P)
    sizes = part.piece_sizes(N, P)
    assert len(blocks) == q * P
    for i in range(P):
        bl = blocks[i * q:(i + 1) * q]
        assert bl[0][0] == starts[i]
        assert sum(b[1] for b in bl) == sizes[i]
        sz = [b[1] for b in bl]
        assert max(sz) - min(sz) <= 1 and sz == sorted(sz, reverse=True)
        for a, b in zip(bl, bl[1:]):
            assert a[0] + a[1] == b[0]
    if N <= 1000:
        R0 = part.restriction_R0(N, P, q).toarray()
        assert np.all(R0.sum(axis=0) == 1)


def test_coarse_rule_values():
    """q = 2^(floor(log2(N/P)) - 4): N/P = 2^S gives 2^(S-4) (Sec. 4.1); capped at N0 <= 16384."""
    assert part.coarse_rule_q(256 * 64, 64) == 16
    assert part.coarse_rule_q(1024 * 8, 8) == 64
    assert part.coarse_rule_q(961, 8) == 4
    assert part.coarse_rule_q(248031, 256) == 32
    assert part.coarse_rule_q(252105, 512) == 16
    assert part.coarse_rule_q(8258175, 4096) == 4      # rule gives 64, cap 16384/4096
    assert part.coarse_rule_q(6885, 16) == 16 and part.coarse_rule_q(11025, 16) == 32
    assert part.coarse_rule_q(20, 8) == 1


def _hilbert_cube_order(d, b):
    n = 1 << b
    pts = np.array(np.meshgrid(*[np.arange(n)] * d, indexing="ij")).reshape(d, -1)
    T = hilbert_transpose([pts[j].astype(np.uint64) for j in range(d)], b)
    keys = np.zeros(pts.shape[1], dtype=np.uint64)
    for lev in range(b - 1, -1, -1):
        for j in range(d):
            keys = (keys << np.uint64(1)) | ((T[j] >> np.uint64(lev)) & np.uint64(1))
    return pts, keys


@pytest.mark.parametrize("d,b", [(2, 1), (2, 4), (3, 3), (4, 2), (5, 2), (6, 2)])
def test_hilbert_is_a_continuous_nested_curve(d, b):
    """Defining properties of a Hilbert curve on the 2^b cube: the index is a
    bijection onto 0 .. 2^(db) - 1, consecutive cells are face neighbours
    (the property that sets it apart from Z-order), and every run of 2^(dk)
    consecutive indices fills one aligned sub-cube of side 2^k."""
    pts, keys = _hilbert_cube_order(d, b)
    n = 1 << b
    assert np.array_equal(np.sort(keys), np.arange(n ** d, dtype=np.uint64))
    P = pts[:, np.argsort(keys)].astype(np.int64)
    assert np.all(np.abs(np.diff(P, axis=1)).sum(axis=0) == 1)
    for k in range(1, b):
        blocks = P.reshape(d, -1, 1 << (d * k)) >> k
        assert np.all(blocks == blocks[:, :, :1])


def test_hilbert_two_dimensional_level_one_and_two():
    """The first-order curve visits the four quadrants as a U; the second
    order curve starts in the corner cell of the first quadrant and ends in the
    corner of the last one, both on the same edge of the square."""
    pts, keys = _hilbert_cube_order(2, 1)
    P = pts[:, np.argsort(keys)].T.tolist()
    assert P[0] == [0, 0] and P[3] in ([1, 0], [0, 1])
    assert sorted(map(tuple, P)) == [(0, 0), (0, 1), (1, 0), (1, 1)]
    pts, keys = _hilbert_cube_order(2, 2)
    P = pts[:, np.argsort(keys)].T
    assert P[0].tolist() == [0, 0]
    end = P[-1].tolist()
    assert end in ([3, 0], [0, 3])


def test_hilbert_grid_keys_unique_and_1d_identity():
    g = Grid(levels=(4, 3, 5))
    k = hilbert_keys(g)
    assert len(np.unique(k)) == g.N
    g1 = Grid(levels=(6,))
    sfc_index, _ = sfc_order(g1, "hilbert")
    assert np.array_equal(sfc_index, np.arange(g1.N))


def _order_within(keys: np.ndarray) -> np.ndarray:
    return np.argsort(keys, kind="stable")


@pytest.mark.parametrize("levels", [(4, 4), (3, 3, 3), (2, 2, 2, 2), (3, 2, 4), (2, 4, 3), (1, 3), (4, 1, 2)])
def test_hilbert_keys_follow_the_cube_curve(levels):
    """hilbert_keys itself on a grid: its order of the interior points equals
    the order that the property-checked cube curve (bijective, face-continuous,
    nested; test above) gives to the same points at their scaled coordinates
    C_j = k_j 2^(nres - l_j), nres = max l_j.  A wrong interleave, bit order or
    scaling in hilbert_keys changes this order."""
    g = Grid(levels=levels)
    nres = max(levels)
    pts, cube_keys = _hilbert_cube_order(g.d, nres)
    side = 1 << nres
    lin = np.zeros(pts.shape[1], dtype=np.int64)
    for j in range(g.d):
        lin = lin * side + pts[j]
    lookup = np.empty(side ** g.d, dtype=np.uint64)
    lookup[lin] = cube_keys
    C = g.coords().astype(np.int64) << np.array([nres - l for l in levels], dtype=np.int64)[None, :]
    lin_g = np.zeros(g.N, dtype=np.int64)
    for j in range(g.d):
        lin_g = lin_g * side + C[:, j]
    want = _order_within(lookup[lin_g])
    got = _order_within(hilbert_keys(g))
    assert np.array_equal(got, want)


def _classic_hilbert_2d(x: np.ndarray, y: np.ndarray, b: int) -> np.ndarray:
    """Index along the classic two-dimensional Hilbert curve of side 2^b
    (the quadrant-by-quadrant construction with a rotation/reflection of the
    remaining low bits after each level), vectorised: at level s the quadrant
    digit is 3 rx XOR ry, and the low bits are reflected when (rx, ry) = (1, 0)
    and transposed whenever ry = 0."""
    x = x.astype(np.int64).copy()
    y = y.astype(np.int64).copy()
    n = 1 << b
    out = np.zeros_like(x)
    s = n >> 1
    while s > 0:
        rx = (x & s) > 0
        ry = (y & s) > 0
        out += s * s * ((3 * rx.astype(np.int64)) ^ ry.astype(np.int64))
        flip = (~ry) & rx
        x = np.where(flip, n - 1 - x, x)
        y = np.where(flip, n - 1 - y, y)
        x, y = np.where(~ry, y, x), np.where(~ry, x, y)
        s >>= 1
    return out


def test_hilbert_keys_two_dimensional_are_the_classic_curve():
    """An independent construction: on the 2^b x 2^b grids (b = 2..6) the
    order hilbert_keys gives the interior points is the order of the classic
    two-dimensional Hilbert curve composed with one fixed symmetry of the
    square (the same symmetry at every b)."""
    found = None
    for b in range(6, 1, -1):
        g = Grid(levels=(b, b))
        K = g.coords().astype(np.int64)
        got = _order_within(hilbert_keys(g))
        n = (1 << b) - 1
        ok = []
        for swap in (False, True):
            for fx in (False, True):
                for fy in (False, True):
                    u = n - K[:, 0] if fx else K[:, 0]
                    v = n - K[:, 1] if fy else K[:, 1]
                    if swap:
                        u, v = v, u
                    if np.array_equal(got, _order_within(_classic_hilbert_2d(u, v, b))):
                        ok.append((swap, fx, fy))
        assert ok, b
        if found is None:
            assert len(ok) == 1
            found = ok[0]
        assert found in ok, (b, ok)
