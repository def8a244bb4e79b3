"""Differentiable solve u = A(a)^{-1} f with a hand-written adjoint backward.

The operator is the FD matrix of -sum_j a_j d^2u/dx_j^2 = f (Sec. 4 model
problem with alpha = diag(a_j)).  A is symmetric, so the adjoint solve reuses
the forward context (same factors):  lambda = A^{-1} dJ/du,  dJ/df = lambda,
dJ/da_j = -lambda^T (dA/da_j) u, the last computed by the library's
coefficient-gradient kernel.
"""
from __future__ import annotations

from fractions import Fraction

import torch


class PoissonSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, a, opts):
        from . import SFCSchwarz
        coeff = [float(v) for v in a.detach().cpu().tolist()]
        solver = SFCSchwarz(coeff=coeff, device=f.device, **opts["setup"])
        u, info = solver.solve(f.detach().contiguous(), **opts["solve"])
        ctx.solver = solver
        ctx.opts = opts
        ctx.a_device = a.device
        ctx.save_for_backward(u)
        ctx.forward_info = info
        return u

    @staticmethod
    def backward(ctx, grad_u):
        (u,) = ctx.saved_tensors
        lam, _ = ctx.solver.solve(grad_u.detach().contiguous(), **ctx.opts["solve"])
        grad_f = lam if ctx.needs_input_grad[0] else None
        grad_a = None
        if ctx.needs_input_grad[1]:
            grad_a = torch.tensor(ctx.solver.grad_coeff(lam, u), dtype=torch.float64,
                                  device=ctx.a_device)
        return grad_f, grad_a, None


def solve_poisson(f, a, levels, P, gamma=Fraction(1, 2), q=0, factor_dtype="fp64",
                  local_solver="cholesky", rtol=1e-12, max_iter=1000, method=None):
    """u = A(a)^{-1} f on the level-`levels` grid, differentiable in f and a."""
    if method is None:
        method = "fcg" if factor_dtype == "fp32" else "pcg"
    opts = {"setup": dict(levels=list(levels), P=P, gamma=gamma, q=q, factor_dtype=factor_dtype,
                          local_solver=local_solver),
            "solve": dict(rtol=rtol, max_iter=max_iter, method=method)}
    return PoissonSolve.apply(f, a, opts)
