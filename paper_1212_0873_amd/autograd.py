"""torch.autograd face of the solver: x(b, lambda) with a hand-written adjoint.

``lasso(problem, b, lam)`` solves min 0.5||A x - b||^2 + lam ||x||_1 for the
matrix held by ``problem`` (a :class:`Problem`), warm-started from its current
x, and returns x as a float64 CUDA tensor.  Its backward calls
``pcdm_grad_backward``: the active-set adjoint solved by the same PCDM kernels.
"""

from __future__ import annotations

import torch

from .api import Problem


class LassoSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, lam, problem: Problem, rel_gap: float):
        problem.set_rhs(b.detach())
        problem.set_option("lambda", float(lam.detach().item()))
        st = problem.solve(rel_gap=rel_gap)
        if not st["converged"]:
            raise RuntimeError(f"forward solve did not reach rel_gap {rel_gap}: {st}")
        ctx.problem = problem
        ctx.lam_meta = (lam.dtype, lam.device)
        return problem.get_x_tensor(torch.float64)

    @staticmethod
    def backward(ctx, grad_x):
        dldb, dldlam = ctx.problem.grad_backward(grad_x.detach())
        dtype, device = ctx.lam_meta
        return dldb, torch.tensor(dldlam, dtype=dtype, device=device), None, None


def lasso(problem: Problem, b: torch.Tensor, lam: torch.Tensor, rel_gap: float = 1e-9) -> torch.Tensor:
    """x(b, lam) as a differentiable function of b (CUDA, float64) and lam (0-d tensor)."""
    return LassoSolve.apply(b, lam, problem, rel_gap)
