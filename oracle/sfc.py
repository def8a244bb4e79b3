"""Z-order space-filling-curve ordering (oracle, test infrastructure).

Sec. 3.3 / Alg. 1 (setup, computation of sfc_index): the interior points are
mapped to the 1-D parameter space of a discrete space-filling curve whose
resolution is that of the finest direction, max_j l_j, and sorted along it.
The curve here is the Z-order (Morton) curve.  Points sit at their geometric
positions x_j = k_j h_j = k_j 2^{-l_j}; on the finest resolution grid this is
the integer coordinate C_j = k_j * 2^(nres - l_j).  The Morton key interleaves
the bits of C_1..C_d, bit b of C_j going to key bit b*d + j (dimension 1 is the
least significant within each bit level).

For explicit point counts n_j (no dyadic embedding) C_j = k_j and
nres = ceil(log2(max_j n_j + 1)).

sfc_index = argsort(keys): sfc_index[p] is the natural index of the point at
curve position p; pos is its inverse.
"""
from __future__ import annotations

import numpy as np

from .grid import Grid


def resolution(g: Grid):
    """(nres, shifts) of the curve: resolution bits and per-dimension scaling."""
    if g.levels is not None:
        nres = max(g.levels)
        shifts = [nres - l for l in g.levels]
    else:
        nres = max(int(np.ceil(np.log2(max(g.n) + 1))), 1)
        shifts = [0] * g.d
    if nres * g.d > 64:
        raise OverflowError("Morton key needs more than 64 bits")
    return nres, shifts


def morton_keys(g: Grid) -> np.ndarray:
    """uint64 Morton key of every point, natural order."""
    nres, shifts = resolution(g)
    K = g.coords().astype(np.uint64)
    keys = np.zeros(g.N, dtype=np.uint64)
    for j in range(g.d):
        C = K[:, j] << np.uint64(shifts[j])
        for b in range(nres):
            bit = (C >> np.uint64(b)) & np.uint64(1)
            keys |= bit << np.uint64(b * g.d + j)
    return keys


def sfc_order(g: Grid):
    """(sfc_index, pos): curve order by sorting the keys (they are unique)."""
    keys = morton_keys(g)
    sfc_index = np.argsort(keys, kind="stable").astype(np.int64)
    if g.N > 1 and not np.all(keys[sfc_index][1:] > keys[sfc_index][:-1]):
        raise AssertionError("Morton keys are not unique")
    pos = np.empty(g.N, dtype=np.int64)
    pos[sfc_index] = np.arange(g.N, dtype=np.int64)
    return sfc_index, pos
