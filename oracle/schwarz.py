"""Two-level overlapping Schwarz preconditioners (oracle, test infrastructure).

Sec. 3.1, 3.3, Alg. 1 and Alg. 2:
  local matrices   A_i = R_i A R_i^T                         (Sec. 3.1)
  factor once      Cholesky of every A_i and of A_0          (Sec. 3.1)
  coarse matrix    A_0 = R_0 A R_0^T                         (eq. csm)
  weighted 1-level C1^{-1} = sum_i R_i^T D_i A_i^{-1} R_i     (eq. w1levprec)
  additive         C^{-1} = R_0^T A_0^{-1} R_0 + C1^{-1}      (eq. addSW, Alg. 2)
  balanced         C^{-1} = G^T C1^{-1} G + F,               (eq. balSW)
                   F = R_0^T A_0^{-1} R_0, G = I - A F        (eq. balan)
  deflated         C^{-1} = G^T C1^{-1} + F                  (Sec. 3.1, after eq. balan)
The coarse right-hand side in Alg. 2 is read as R_0 g (the input vector).
Vectors passed in and out are in natural order; internally everything is in
curve-position order (row p of the permuted matrix is the point sfc_index[p]).
"""
from __future__ import annotations

from fractions import Fraction
from typing import Optional, Sequence

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .grid import Grid
from . import partition as part
from .sfc import sfc_order

WEIGHT_NONE, WEIGHT_OMEGA, WEIGHT_D = "none", "omega", "D"


class OracleSchwarz:
    def __init__(self, grid: Grid, P: int, gamma, q: Optional[int] = None,
                 weighting: str = WEIGHT_OMEGA, variant: str = "balanced",
                 factor: bool = True, curve: str = "zorder"):
        self.g = grid
        self.N = grid.N
        self.P = int(P)
        self.gamma = Fraction(gamma)
        if not (1 <= self.P <= self.N):
            raise ValueError("need 1 <= P <= N")
        self.q = part.coarse_rule_q(self.N, self.P) if q is None else int(q)
        self.weighting = weighting
        self.variant = variant
        self.curve = curve
        self.sfc_index, self.pos = sfc_order(grid, curve)
        A_nat = grid.matrix()
        perm = self.sfc_index
        self.A_nat = A_nat
        self.A = A_nat[perm][:, perm].tocsr()          # curve-position order
        self.sets = part.overlap_sets(self.N, self.P, self.gamma)
        rng = [part.cyclic_range(S, self.N) for S in self.sets]
        self.ta = np.array([r[0] for r in rng], dtype=np.int64)
        self.Ni = np.array([r[1] for r in rng], dtype=np.int64)
        self.orders = [r[2] for r in rng]
        self.mult = part.multiplicity(self.sets, self.N)
        self.omega = part.omega(self.sets, self.mult)
        self.R0 = part.restriction_R0(self.N, self.P, self.q)
        self.A0 = (self.R0 @ self.A @ self.R0.T).toarray()
        self.local = None
        if factor:
            self.factor()

    # -- setup ---------------------------------------------------------
    def local_matrix(self, i: int) -> np.ndarray:
        """A_i = R_i A R_i^T in the subdomain's local (cyclic curve) order."""
        o = self.orders[i]
        return self.A[o][:, o].toarray()

    def factor(self):
        self.local = [sla.cho_factor(self.local_matrix(i), lower=True) for i in range(self.P)]
        self.coarse = sla.cho_factor(self.A0, lower=True)

    def weights(self, i: int) -> np.ndarray:
        if self.weighting == WEIGHT_NONE:
            return np.ones(int(self.Ni[i]))
        if self.weighting == WEIGHT_OMEGA:
            return np.full(int(self.Ni[i]), self.omega[i])
        if self.weighting == WEIGHT_D:
            return 1.0 / self.mult[self.orders[i]]
        raise ValueError(self.weighting)

    # -- operators in curve order ----------------------------------------
    def local_solve(self, i: int, g_s: np.ndarray) -> np.ndarray:
        """d_i = A_i^{-1} R_i g (Alg. 2, first two steps)."""
        return sla.cho_solve(self.local[i], g_s[self.orders[i]])

    def fine_s(self, g_s: np.ndarray) -> np.ndarray:
        """C1^{-1} g = sum_i R_i^T D_i A_i^{-1} R_i g (eq. w1levprec)."""
        h = np.zeros(self.N)
        for i in range(self.P):
            np.add.at(h, self.orders[i], self.weights(i) * self.local_solve(i, g_s))
        return h

    def coarse_s(self, g_s: np.ndarray) -> np.ndarray:
        """F g = R_0^T A_0^{-1} R_0 g (eq. balan)."""
        d0 = sla.cho_solve(self.coarse, self.R0 @ g_s)
        return self.R0.T @ d0

    def apply_s(self, g_s: np.ndarray) -> np.ndarray:
        if self.variant == "additive":
            return self.coarse_s(g_s) + self.fine_s(g_s)
        if self.variant == "balanced":
            t = self.coarse_s(g_s)                 # F g
            w = g_s - self.A @ t                   # G g
            y = self.fine_s(w)                     # C1^{-1} G g
            s = self.coarse_s(self.A @ y)          # F A y
            return y - s + t                       # G^T y + F g
        if self.variant == "deflated":
            t = self.coarse_s(g_s)                 # F g
            y = self.fine_s(g_s)                   # C1^{-1} g
            s = self.coarse_s(self.A @ y)          # F A y
            return y - s + t                       # G^T C1^{-1} g + F g
        if self.variant == "onelevel":
            return self.fine_s(g_s)
        raise ValueError(self.variant)

    # -- natural-order interface -------------------------------------------
    def to_s(self, v):
        return np.asarray(v, dtype=np.float64)[self.sfc_index]

    def from_s(self, v_s):
        out = np.empty(self.N)
        out[self.sfc_index] = v_s
        return out

    def apply(self, g: np.ndarray) -> np.ndarray:
        """h = C^{-1} g, natural order in and out."""
        return self.from_s(self.apply_s(self.to_s(g)))

    def matvec(self, x: np.ndarray) -> np.ndarray:
        return self.A_nat @ x

    def balancing_start(self, b: np.ndarray, x0: Optional[np.ndarray] = None) -> np.ndarray:
        """x0 + F (b - A x0) in natural order: the coarse-corrected start of
        the balanced iteration (F = R_0^T A_0^{-1} R_0, eq. balan).  Its
        residual r satisfies R_0 r = R_0 b - A_0 A_0^{-1} R_0 b = 0 (for x0 = 0),
        and since R_0 A C^{-1} r = R_0 r for the balanced C^{-1}, CG and
        Richardson keep R_0 r_k = 0 from there on."""
        x = np.zeros(self.N) if x0 is None else np.asarray(x0, dtype=np.float64)
        r_s = self.to_s(b - self.A_nat @ x)
        return x + self.from_s(self.coarse_s(r_s))

    def dense_preconditioner(self) -> np.ndarray:
        """C^{-1} as a dense matrix in natural order (tiny grids only)."""
        I = np.eye(self.N)
        return np.column_stack([self.apply(I[:, k]) for k in range(self.N)])
