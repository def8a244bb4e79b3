"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds input generation only: a counter-based random generator
(splitmix64, as published by Steele, Lea and Flood, 2014), the workload
descriptions (grid levels, subdomain counts, overlap parameters, seeds) and
the manufactured test problem of the combination-technique study.  It
contains none of the solver's arithmetic, so the oracle and the library can
both draw the same right-hand sides and coefficients without sharing any
method code.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction
from itertools import product
from typing import List, Optional, Tuple

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Outputs offset+1 .. offset+n of splitmix64 started from state `seed`.

    Output k (1-based) mixes the state seed + k * 0x9E3779B97F4A7C15 (mod 2^64).
    """
    k = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int) -> np.ndarray:
    """n doubles in [0, 1): the top 53 bits of each splitmix64 output."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_pm1(seed: int, n: int) -> np.ndarray:
    """n doubles in [-1, 1): 2u - 1 with u from `uniform01` (exact in binary64)."""
    return 2.0 * uniform01(seed, n) - 1.0


def log_uniform_coeff(seed: int, d: int, lo_exp: float = -1.0, hi_exp: float = 1.0) -> np.ndarray:
    """d diffusion coefficients 10^(lo + (hi-lo) u), log-uniform on [10^lo, 10^hi]."""
    u = uniform01(seed, d)
    return 10.0 ** (lo_exp + (hi_exp - lo_exp) * u)


def ct_levels(d: int, total: int, lmin: int) -> List[Tuple[int, ...]]:
    """All level vectors l in N^d with |l|_1 = total and every l_j >= lmin,
    in lexicographic order."""
    out = []
    for l in product(range(lmin, total + 1), repeat=d):
        if sum(l) == total:
            out.append(tuple(l))
    return out


def manufactured(x: np.ndarray):
    """(u, f) of Sec. 4.3 at points x (M, d): u = |x| prod sin(pi x_j),
    f = -Laplace(u) = -(s (d-1)/r + (2 pi / r) sum_i x_i cos(pi x_i) prod_{j!=i} sin(pi x_j)
    - d pi^2 r s), r = |x|, s = prod sin(pi x_j)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    d = x.shape[1]
    r = np.sqrt((x * x).sum(axis=1))
    sn = np.sin(np.pi * x)
    s = np.prod(sn, axis=1)
    grad_term = np.zeros(x.shape[0])
    for i in range(d):
        others = np.prod(np.delete(sn, i, axis=1), axis=1) if d > 1 else np.ones(x.shape[0])
        grad_term += x[:, i] * np.pi * np.cos(np.pi * x[:, i]) * others
    lap = s * (d - 1) / r + 2.0 * grad_term / r - d * np.pi ** 2 * r * s
    return r * s, -lap


@dataclass
class Workload:
    """One synthetic workload: the grid(s), partition parameters and seeds."""
    name: str
    levels: List[Tuple[int, ...]]          # one level vector per grid
    P: int                                  # subdomains per grid
    gamma: Fraction                         # overlap parameter
    seeds: List[int]                        # right-hand-side seed per grid
    rtol: float
    coeff: Optional[List[float]] = None     # diffusion coefficients a_j (None: all 1)
    note: str = ""

    @property
    def d(self) -> int:
        return len(self.levels[0])

    def npts(self, g: int = 0) -> List[int]:
        return [(1 << l) - 1 for l in self.levels[g]]

    def N(self, g: int = 0) -> int:
        return int(np.prod(self.npts(g)))

    def rhs(self, g: int = 0) -> np.ndarray:
        """f iid U[-1,1) in natural order (first coordinate fastest)."""
        return uniform_pm1(self.seeds[g], self.N(g))


def workloads() -> dict:
    """The five workloads the solver is exercised on."""
    c3_coeff = [float(v) for v in log_uniform_coeff(1003, 6)]
    c4_lv = ct_levels(4, 14, 2)
    return {
        # d=2, 31x31, P=8, 50% overlap (gamma = 1/4), rtol 1e-10
        "c1": Workload("d2_l5x5_P8", [(5, 5)], 8, Fraction(1, 4), [1], 1e-10),
        # d=3 anisotropic 127x63x31, P=256, 100% overlap (gamma = 1/2)
        "c2": Workload("d3_l7x6x5_P256", [(7, 6, 5)], 256, Fraction(1, 2), [2], 1e-9),
        # d=6, 7^5 x 15, P=512, 50% overlap, log-uniform coefficients
        "c3": Workload("d6_l333334_P512", [(3, 3, 3, 3, 3, 4)], 512, Fraction(1, 4), [3], 1e-9,
                       coeff=c3_coeff),
        # d=4 combination-technique layer |l|_1 = 14, l_j >= 2: 84 grids, P=16 each
        "c4": Workload("d4_ct14_84grids_P16", c4_lv, 16, Fraction(1, 4),
                       [4000 + g for g in range(len(c4_lv))], 1e-9),
        # d=3, 255x255x127, P=4096, 25% overlap (gamma = 1/8)
        "c5": Workload("d3_l8x8x7_P4096", [(8, 8, 7)], 4096, Fraction(1, 8), [5], 1e-9),
    }
