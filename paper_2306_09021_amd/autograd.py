"""torch.autograd.Function around pbng_solve (forward) and pbng_adjoint
(backward): the equilibrium x*(x_D, mu, lambda) as a differentiable function
of the Dirichlet targets and the per-tet Lame parameters.  Marshalling only:
the solve, the adjoint solve and the gradient assembly run in libpbng."""
from __future__ import annotations

import torch

from . import pbng


class Equilibrium(torch.autograd.Function):
    """x = Equilibrium.apply(x_D, mu, lam, ws, x_init, solve_opts, adjoint_opts)

    x_D: float64 cuda [n_dirichlet, 3] (creation order), mu / lam: float64
    cuda [n_tets]; x_init: cuda [n_verts, 3] of the workspace dtype.  Returns
    the equilibrium positions (workspace dtype).  The backward pass solves
    the adjoint system by block Gauss-Seidel on the true Hessian and returns
    dL/dx_D (including the direct term of the Dirichlet rows), dL/dmu and
    dL/dlambda."""

    @staticmethod
    def forward(ctx, x_D, mu, lam, ws, x_init, solve_opts, adjoint_opts):
        ws.set_dirichlet(x_D.detach().contiguous())
        ws.set_materials(mu.detach().contiguous(), lam.detach().contiguous())
        x = x_init.detach().clone().contiguous()
        rc, st = ws.solve(x, solve_opts)
        ctx.ws = ws
        ctx.adjoint_opts = adjoint_opts
        ctx.stats = st
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, grad_x):
        (x,) = ctx.saved_tensors
        g = grad_x.detach().to(x.dtype).contiguous()
        rc, out, st = ctx.ws.adjoint(x, g, ctx.adjoint_opts, want=("xd", "mu", "lam"))
        ctx.adjoint_stats = st
        return out["xd"], out["mu"], out["lam"], None, None, None, None


def equilibrium(x_D, mu, lam, ws, x_init, solve_opts=None, adjoint_opts=None):
    so = solve_opts if solve_opts is not None else pbng.solve_opts()
    ao = adjoint_opts if adjoint_opts is not None else pbng.adjoint_opts()
    return Equilibrium.apply(x_D, mu, lam, ws, x_init, so, ao)
