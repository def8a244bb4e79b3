"""Combination technique on top of the batched solver (Sec. 2).

All full grids of the combination technique of level L in d dimensions are
set up as one batch: the grids of layer i (|l|_1 = L + d - 1 - i, l_j >= 1,
i = 0 .. d-1) get P = Phat 2^(d-1-i) subdomains (eq. Pchoice; at most the
grid's size) and the weight (-1)^i binom(d-1, i) (eq. combi).  The grids are
independent, so one setup and one solve cover all of them; the combined
solution is evaluated at arbitrary points by the library's combination
kernel (multilinear evaluation of every grid, summed in a fixed order).  The
layout (level vectors, layers, weights, subdomain counts) comes from the
library's sfcdd_ct_layout; this module only marshals.
"""
from __future__ import annotations

import ctypes
from fractions import Fraction

import numpy as np


def ct_layout(d: int, L: int, phat: int = 1):
    """[(level vector, layer i, weight, P)] of the level-L combination in d
    dimensions, from the library's sfcdd_ct_layout (layers |l|_1 = L + d - 1 - i,
    weight (-1)^i binom(d-1, i), P = Phat 2^(d-1-i) capped at the grid's
    size)."""
    from . import _check, lib
    n = ctypes.c_int32()
    _check(lib().sfcdd_ct_layout(int(d), int(L), int(phat), 0, ctypes.byref(n), None, None, None, None))
    G = n.value
    lv = (ctypes.c_int32 * (G * d))()
    lay = (ctypes.c_int32 * G)()
    w = (ctypes.c_double * G)()
    P = (ctypes.c_int32 * G)()
    _check(lib().sfcdd_ct_layout(int(d), int(L), int(phat), G, ctypes.byref(n), lv, lay, w, P))
    return [(tuple(lv[k * d:(k + 1) * d]), int(lay[k]), float(w[k]), int(P[k])) for k in range(G)]


class CombinationTechnique:
    def __init__(self, d: int, L: int, phat: int = 1, gamma=Fraction(1, 4), factor_dtype: str = "fp32",
                 variant: str = "balanced", weighting: str = "omega", curve: str = "zorder",
                 layout: str = "natural", device="cuda:0", workspace=None):
        import torch
        from . import SFCSchwarzBatch
        if d < 1 or L < 1:
            raise ValueError("need d >= 1 and L >= 1")
        self.d, self.L = d, L
        self.levels, self.layer, self.weights, grids = [], [], [], []
        for lv, i, w, P in ct_layout(d, L, phat):
            self.levels.append(lv)
            self.layer.append(i)
            self.weights.append(w)
            grids.append(dict(levels=list(lv), P=P, gamma=gamma, curve=curve))
        self.batch = SFCSchwarzBatch(grids, factor_dtype=factor_dtype, variant=variant,
                                     weighting=weighting, layout=layout, device=device,
                                     workspace=workspace)
        self.device = self.batch.device
        self.weights_dev = torch.tensor(self.weights, dtype=torch.float64, device=self.device)
        self.method = "fcg" if factor_dtype == "fp32" else "pcg"

    @property
    def ngrids(self) -> int:
        return len(self.levels)

    @property
    def total_unknowns(self) -> int:
        return self.batch.N

    def grid_points(self, g: int) -> np.ndarray:
        """(N_g, d) coordinates k_j / (n_j + 1) of grid g's points, natural
        order (first coordinate fastest)."""
        n = [(1 << l) - 1 for l in self.levels[g]]
        axes = [np.arange(1, nj + 1) / (nj + 1) for nj in n]
        mesh = np.meshgrid(*reversed(axes), indexing="ij")
        return np.stack([m.reshape(-1) for m in reversed(mesh)], axis=1)

    def solve(self, f, rtol=1e-8, max_iter=1000, method=None, recursive=True):
        """Solutions of all grids for the concatenated right-hand sides f
        (device tensor, grid after grid, each in the context's layout).  The
        default stopping test is the one of Sec. 4.3, the relative recursive
        residual of every grid below rtol: on the grids with 2^(L+d-1)
        points along one axis the true residual has a rounding floor near
        1e-8 in FP64."""
        return self.batch.solve(f, rtol=rtol, max_iter=max_iter, method=method or self.method,
                                recursive=recursive)

    def evaluate(self, u, x):
        """u^(c)(x) at the points x (contiguous float64 device tensor (M, d))
        for the concatenated grid solutions u; points outside [0, 1]^d are
        extrapolated from the boundary cells."""
        import torch
        from . import _check, lib
        if not isinstance(x, torch.Tensor) or x.dtype != torch.float64 or x.device != self.device \
                or x.dim() != 2 or x.shape[1] != self.d or not x.is_contiguous():
            raise ValueError(f"x must be a contiguous float64 (M, {self.d}) tensor on {self.device}")
        M = x.shape[0]
        out = torch.empty(M, dtype=torch.float64, device=self.device)
        _check(lib().sfcdd_ct_combine(self.batch.ctx, ctypes.c_void_p(self.weights_dev.data_ptr()),
                                      self.batch._vec(u, "u"), ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_int64(M), ctypes.c_void_p(out.data_ptr())), self.batch.ctx)
        return out

    def close(self):
        self.batch.close()
