"""torch.autograd wrapper: V = orthonormal basis of null(A) as a function of A's values.

The forward pass loads the values into a :class:`Context` built for A's
pattern (``nullspace_update_values``), runs the solver and returns V (n x N).
The backward pass hands dL/dV to the library's ``backward`` entry point (range
CG on A^T A plus the SDDMM) and returns dL/dvals in A's CSR order.

V is unique only up to a rotation of its columns, so the loss must depend on V
through the projector P = V V^T alone (e.g. ||V^T X||_F^2 or tr(P M)); then
dL/dV = 2 G_s V with G_s the symmetric part of dL/dP, and the library takes
G_s V = dL/dV / 2.  N is held fixed: the derivative is that of the projector
onto the N smallest right singular vectors, defined while sigma_{N+1} > 0.

One solve per Context at a time: a forward pass replaces the Context's basis,
so a backward pass must run before the next forward pass on the same Context
(checked).
"""
from __future__ import annotations

import torch

from ._lib import Context


class NullSpaceFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals: torch.Tensor, solver: Context, tol: float, max_iter: int):
        solver.update_values(vals.detach().contiguous())
        solver.lanczos_run()
        solver._generation = getattr(solver, "_generation", 0) + 1
        ctx.solver = solver
        ctx.generation = solver._generation
        ctx.tol, ctx.max_iter = tol, max_iter
        return solver.extract_basis().contiguous()

    @staticmethod
    def backward(ctx, grad_v: torch.Tensor):
        solver = ctx.solver
        if getattr(solver, "_generation", 0) != ctx.generation:
            raise RuntimeError("the Context ran another forward pass before this backward pass")
        grad, _ = solver.backward(grad_v.contiguous(), tol=ctx.tol, max_iter=ctx.max_iter)
        return grad, None, None, None


def null_space(vals: torch.Tensor, solver: Context, tol: float = 1e-10,
               max_iter: int = 10 ** 6) -> torch.Tensor:
    """Differentiable V (n x N) for the values ``vals`` (nnz, float64, CUDA) of the
    pattern ``solver`` was built with; see the module docstring for the loss
    requirement.  ``tol`` and ``max_iter`` go to the backward CG."""
    return NullSpaceFunction.apply(vals, solver, tol, max_iter)
