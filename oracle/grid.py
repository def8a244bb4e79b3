"""Model problem and its finite-difference matrix (oracle, test infrastructure).

Sec. 3.3 (eq. dof): N = prod_j (2^{l_j} - 1) interior points of the grid with
mesh widths h_j = 2^{-l_j}.  Sec. 4: -div(alpha grad u) = f on [0,1]^d with
homogeneous Dirichlet data; here alpha = diag(a_1..a_d) is constant,
discretised by the (2d+1)-point finite-difference stencil scaled by 1/h_j^2
(the scaling under which the level (m,1,...,1) grid reduces to the 1-D
operator plus 8(d-1) I, Sec. 4.2).

Natural ordering: point k = (k_1..k_d), 1 <= k_j <= n_j, has natural index
sum_j (k_j - 1) * stride_j with the first coordinate fastest.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence

import numpy as np
import scipy.sparse as sp


class Grid:
    """Interior grid of one (possibly anisotropic) subproblem.

    levels: level vector l (n_j = 2^{l_j} - 1, h_j = 2^{-l_j}), or
    npts:   explicit point counts n_j (h_j = 1/(n_j + 1)), used for the 1-D
            weak-scaling experiments where N = 2^S P is not of the form 2^l - 1.
    coeff:  diffusion coefficients a_j (default all 1).
    """

    def __init__(self, levels: Optional[Sequence[int]] = None,
                 npts: Optional[Sequence[int]] = None,
                 coeff: Optional[Sequence[float]] = None):
        if (levels is None) == (npts is None):
            raise ValueError("give exactly one of levels / npts")
        if levels is not None:
            self.levels = [int(l) for l in levels]
            self.n = [(1 << l) - 1 for l in self.levels]
        else:
            self.levels = None
            self.n = [int(v) for v in npts]
        self.d = len(self.n)
        self.a = [1.0] * self.d if coeff is None else [float(v) for v in coeff]
        # 1/h_j^2 = (n_j + 1)^2 exactly; c_j = a_j / h_j^2
        self.inv_h2 = [float((nj + 1) * (nj + 1)) for nj in self.n]
        self.c = [self.a[j] * self.inv_h2[j] for j in range(self.d)]
        self.N = int(np.prod(self.n))
        self.stride = [int(np.prod(self.n[:j])) for j in range(self.d)]

    def coords(self) -> np.ndarray:
        """(N, d) int64 array of 1-based grid coordinates in natural order."""
        nat = np.arange(self.N, dtype=np.int64)
        k = np.empty((self.N, self.d), dtype=np.int64)
        for j in range(self.d):
            k[:, j] = (nat // self.stride[j]) % self.n[j] + 1
        return k

    def second_difference(self, j: int) -> sp.csr_matrix:
        """Integer matrix L_j = tridiag(-1, 2, -1) along dimension j, identity
        across the others (Dirichlet neighbours dropped)."""
        T = sp.diags([-np.ones(self.n[j] - 1), 2 * np.ones(self.n[j]), -np.ones(self.n[j] - 1)],
                     [-1, 0, 1], format="csr")
        # kron order: the last factor varies fastest, i.e. dimension 0 last.
        M = sp.identity(1, format="csr")
        for jj in reversed(range(self.d)):
            M = sp.kron(M, T if jj == j else sp.identity(self.n[jj], format="csr"), format="csr")
        return M

    def matrix(self) -> sp.csr_matrix:
        """A = sum_j (a_j / h_j^2) L_j, the (2d+1)-point FD matrix (SPD)."""
        A = None
        for j in range(self.d):
            term = self.c[j] * self.second_difference(j)
            A = term if A is None else A + term
        return A.tocsr()

    def eigen(self, kvec: Sequence[int]):
        """Closed-form eigenpair of A: v_k(x) = prod_j sin(k_j pi x_j),
        lambda_k = sum_j 4 c_j sin^2(k_j pi / (2 (n_j + 1)))."""
        K = self.coords()
        v = np.ones(self.N)
        lam = 0.0
        for j in range(self.d):
            v *= np.sin(kvec[j] * np.pi * K[:, j] / (self.n[j] + 1))
            lam += 4.0 * self.c[j] * math.sin(kvec[j] * math.pi / (2 * (self.n[j] + 1))) ** 2
        return v, lam
