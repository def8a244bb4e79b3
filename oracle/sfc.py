"""Z-order and Hilbert space-filling-curve orderings (oracle, test infrastructure).

Sec. 3.3 / Alg. 1 (setup, computation of sfc_index): the interior points are
mapped to the 1-D parameter space of a discrete space-filling curve whose
resolution is that of the finest direction, max_j l_j, and sorted along it.
Two curves: Z-order (Morton) and Hilbert (the paper's choice, Sec. 3.2).
Points sit at their geometric positions x_j = k_j h_j = k_j 2^{-l_j}; on the
finest resolution grid this is the integer coordinate C_j = k_j * 2^(nres - l_j).
The Morton key interleaves the bits of C_1..C_d, bit b of C_j going to key bit
b*d + j (dimension 1 is the least significant within each bit level).  The
Hilbert key is Skilling's transposed index of (C_1..C_d) read level by level
from the top, dimension 1 first (see hilbert_transpose).

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


def hilbert_transpose(X, nres: int):
    """Skilling's axes-to-transposed-index transform of the Hilbert curve
    (Skilling 2004, the construction the paper's curve references build on),
    vectorised over points.  X: list of d uint64 arrays of nres-bit
    coordinates; returns the d arrays T_0..T_{d-1} whose bits, read level by
    level from the top with T_0 first, are the Hilbert index.

    Steps: from the top bit level down, for each axis i, if axis i has a 1 at
    this level the lower bits of axis 0 are inverted, otherwise the lower bits
    of axes 0 and i are exchanged; then the axes are Gray-coded (each XORed
    with the previous one) and the lower bits of every axis are inverted once
    for every 1 that the last Gray-coded axis has at a higher level."""
    d = len(X)
    X = [np.asarray(x, dtype=np.uint64).copy() for x in X]
    one = np.uint64(1)
    for lev in range(nres - 1, 0, -1):
        Q = one << np.uint64(lev)
        low = Q - one
        for i in range(d):
            hit = (X[i] & Q) != 0
            X[0] = np.where(hit, X[0] ^ low, X[0])
            swap = np.where(hit, np.uint64(0), (X[0] ^ X[i]) & low)
            X[0] = X[0] ^ swap
            X[i] = X[i] ^ swap
    for i in range(1, d):
        X[i] = X[i] ^ X[i - 1]
    flip = np.zeros_like(X[0])
    for lev in range(nres - 1, 0, -1):
        Q = one << np.uint64(lev)
        flip = np.where((X[d - 1] & Q) != 0, flip ^ (Q - one), flip)
    return [x ^ flip for x in X]


def hilbert_keys(g: Grid) -> np.ndarray:
    """uint64 Hilbert index of every point, natural order: Skilling's
    transform of the scaled coordinates C_j at resolution nres, bits
    interleaved level by level from the top, dimension 1 (T_0) first."""
    nres, shifts = resolution(g)
    K = g.coords().astype(np.uint64)
    X = [K[:, j] << np.uint64(shifts[j]) for j in range(g.d)]
    T = hilbert_transpose(X, nres)
    keys = np.zeros(g.N, dtype=np.uint64)
    for b in range(nres - 1, -1, -1):
        for j in range(g.d):
            keys = (keys << np.uint64(1)) | ((T[j] >> np.uint64(b)) & np.uint64(1))
    return keys


def sfc_order(g: Grid, curve: str = "zorder"):
    """(sfc_index, pos): curve order by sorting the keys (they are unique)."""
    keys = morton_keys(g) if curve == "zorder" else hilbert_keys(g)
    sfc_index = np.argsort(keys, kind="stable").astype(np.int64)
    if g.N > 1 and not np.all(keys[sfc_index][1:] > keys[sfc_index][:-1]):
        raise AssertionError("curve keys are not unique")
    pos = np.empty(g.N, dtype=np.int64)
    pos[sfc_index] = np.arange(g.N, dtype=np.int64)
    return sfc_index, pos
