"""Disjoint pieces, overlapping subdomains, weights and coarse blocks
(oracle, test infrastructure).  All indices are 0-based curve positions.

Readings of the paper taken here (each also listed in the design notes):
  * overlap parameter gamma is an exact rational;
  * in the eta-parts of eq. (enlarge) the size N_k is the piece size ~N_k;
  * enumeration of pieces is cyclic (Sec. 3.3, after eq. enlarge), so an
    enlarged set may wrap around the end of the curve; when the union covers
    every point the subdomain is the whole grid, stored from position 0;
  * the local order of a subdomain is its cyclic curve order from its first
    position ta_i (Alg. 1 stores each subdomain as a start and an end in
    sfc_index).
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import List, Tuple

import numpy as np
import scipy.sparse as sp


def piece_sizes(N: int, P: int) -> np.ndarray:
    """eq. (sloc): the first r = N - P floor(N/P) pieces get floor(N/P) + 1
    points, the other P - r get floor(N/P)."""
    base, r = divmod(N, P)
    return np.array([base + 1 if i < r else base for i in range(P)], dtype=np.int64)


def piece_starts(N: int, P: int) -> np.ndarray:
    """First curve position of each piece: the pieces are consecutive."""
    s = piece_sizes(N, P)
    return np.concatenate([[0], np.cumsum(s)[:-1]]).astype(np.int64)


def _piece(N: int, P: int, k: int) -> np.ndarray:
    k %= P
    st = piece_starts(N, P)[k]
    return np.arange(st, st + piece_sizes(N, P)[k], dtype=np.int64)


def overlap_sets(N: int, P: int, gamma: Fraction) -> List[np.ndarray]:
    """eq. (enlarge): Omega_i = ~Omega_i, plus the floor(gamma) whole pieces on
    either side, plus the last ceil(eta ~N_k) points of piece k = i-floor(gamma)-1
    and the first floor(eta ~N_k) points of piece k = i+floor(gamma)+1, with
    eta = gamma - floor(gamma) and piece indices taken modulo P.
    Returned as sorted arrays of curve positions (set semantics)."""
    gamma = Fraction(gamma)
    if gamma < 0:
        raise ValueError("gamma must be >= 0")
    F = math.floor(gamma)
    eta = gamma - F
    sizes = piece_sizes(N, P)
    out = []
    for i in range(P):
        parts = [_piece(N, P, i)]
        for k in range(1, F + 1):
            parts.append(_piece(N, P, i - k))
            parts.append(_piece(N, P, i + k))
        kl = (i - F - 1) % P
        kr = (i + F + 1) % P
        nl = math.ceil(eta * int(sizes[kl]))      # last ceil(eta ~N_kl) of the left piece
        nr = math.floor(eta * int(sizes[kr]))     # first floor(eta ~N_kr) of the right piece
        left = _piece(N, P, kl)
        right = _piece(N, P, kr)
        if nl > 0:
            parts.append(left[len(left) - nl:])
        if nr > 0:
            parts.append(right[:nr])
        out.append(np.unique(np.concatenate(parts)))
    return out


def cyclic_range(S: np.ndarray, N: int) -> Tuple[int, int, np.ndarray]:
    """(ta, Ni, order) of a set that is contiguous along the cyclic curve:
    ta is the position whose predecessor is not in the set (0 for the whole
    grid), order[s] = (ta + s) mod N.  Raises if the set is not one cyclic run."""
    Ni = len(S)
    if Ni == N:
        return 0, N, np.arange(N, dtype=np.int64)
    member = np.zeros(N, dtype=bool)
    member[S] = True
    starts = [int(p) for p in S if not member[(p - 1) % N]]
    if len(starts) != 1:
        raise AssertionError("subdomain is not a single cyclic run")
    ta = starts[0]
    order = (ta + np.arange(Ni, dtype=np.int64)) % N
    if not np.all(member[order]):
        raise AssertionError("subdomain is not contiguous")
    return ta, Ni, order


def multiplicity(sets: List[np.ndarray], N: int) -> np.ndarray:
    """m_p = number of subdomains containing curve position p."""
    m = np.zeros(N, dtype=np.int64)
    for S in sets:
        m[S] += 1
    return m


def point_weights(sets, mult):
    """eq. (Di): (D_i)_pp = 1 / m_p for each p in Omega_i."""
    return [1.0 / mult[S] for S in sets]


def omega(sets, mult) -> np.ndarray:
    """eq. (omegai): omega_i = max over p in Omega_i of (D_i)_pp = 1 / min m_p."""
    return np.array([1.0 / int(mult[S].min()) for S in sets])


def coarse_rule_q(N: int, P: int, cap_n0: int = 16384) -> int:
    """Coarse points per subdomain: the paper's four-levels-coarser rule
    q = 2^(floor(log2(N/P)) - 4) (Sec. 4.1 q = 2^(S-4); Sec. 4.2/4.3
    q = 2^(floor(log2(N/P)) - 4)), at least 1, at most floor(N/P), and capped so
    that the dense coarse problem N0 = qP stays at most cap_n0."""
    base = N // P
    e = max(0, int(math.floor(math.log2(N / P))) - 4) if base >= 1 else 0
    q = 1 << e
    q = min(q, max(1, cap_n0 // P))
    return max(1, min(q, base))


def coarse_blocks(N: int, P: int, q: int) -> List[Tuple[int, int]]:
    """eq. (restr): piece i is split into q consecutive blocks ~Omega_{i,m},
    the first (~N_i mod q) of size floor(~N_i/q)+1, the rest floor(~N_i/q).
    Returns (start, size) of coarse unknown i*q + m."""
    if not (1 <= q <= N // P):
        raise ValueError("need 1 <= q <= floor(N/P)")
    sizes = piece_sizes(N, P)
    starts = piece_starts(N, P)
    out = []
    for i in range(P):
        base, r = divmod(int(sizes[i]), q)
        s = int(starts[i])
        for m in range(q):
            sz = base + 1 if m < r else base
            out.append((s, sz))
            s += sz
    return out


def restriction_R0(N: int, P: int, q: int) -> sp.csr_matrix:
    """R_0 in curve-position space: (R_0)_{iq+m, p} = 1 iff p in ~Omega_{i,m}."""
    rows, cols = [], []
    for I, (s, sz) in enumerate(coarse_blocks(N, P, q)):
        rows.extend([I] * sz)
        cols.extend(range(s, s + sz))
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(q * P, N))
