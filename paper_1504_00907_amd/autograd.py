"""Differentiable DDG-PCG solve for the cell-centred diffusion operator.

u = A(exp(theta))^{-1} f.  The forward pass assembles A on the device
(``ddg_stencil_assemble``), refactors the handle (Galerkin product, coarse
inverse, local factors) and solves.  The backward pass reuses the same
handle for the adjoint solve A lam = dL/du -- A and the two-level
preconditioner are both symmetric, so no transposed operator is needed --
and evaluates dL/dtheta_c = -kappa_c lam^T (dA/dkappa_c) u per cell with
``ddg_stencil_coeff_grad``; dL/df = lam.
"""

from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from .solver import DDGSolver, stencil_assemble, stencil_coeff_grad
from .stencil import cc_pattern


class DiffusionSolver:
    """DDG handle for a fixed cell grid and partition; values follow theta.

    dims = (nx, ny, nz); F (n x k generating vectors) and part (n,) are host
    arrays; theta0 (device float64) supplies the values used for the first
    setup.
    """

    def __init__(self, dims, F: np.ndarray, part: np.ndarray, n_parts: int, overlap: int,
                 theta0: torch.Tensor, precision: str = "fp64", rtol: float = 1e-10,
                 max_iter: int = 1000, bc: str = "dirichlet", **kw):
        self.dims = tuple(int(d) for d in dims)
        self.bc = bc
        self.n = int(np.prod(self.dims))
        self.row_ptr, self.col_idx = cc_pattern(self.dims)
        self.nnz = int(self.row_ptr[-1])
        val = torch.empty(self.nnz, dtype=torch.float64, device=theta0.device)
        stencil_assemble(self.dims, theta0.contiguous(), val, bc=bc)
        torch.cuda.current_stream().synchronize()
        self.solver = DDGSolver(self.n, self.row_ptr, self.col_idx, val.cpu().numpy(), F, part, n_parts,
                                overlap, precision=precision, rtol=rtol, max_iter=max_iter, **kw)
        self.val = val
        self.theta = theta0.detach().clone()   # coefficients of the current factorisation
        self.last_info = {}

    def refactor(self, theta: torch.Tensor):
        stencil_assemble(self.dims, theta, self.val, bc=self.bc)
        self.solver.refactor(self.val)
        self.theta = theta.detach().clone()

    def ensure(self, theta: torch.Tensor):
        """Refactor unless the handle already holds A(exp(theta))."""
        if not torch.equal(self.theta, theta):
            self.refactor(theta)

    def solve(self, f: torch.Tensor, u: Optional[torch.Tensor] = None):
        u, info = self.solver.solve(f, u)
        self.last_info = info
        return u

    def coeff_grad(self, theta, u, lam):
        return stencil_coeff_grad(self.dims, theta, u, lam, bc=self.bc)


class DDGSolveFunction(torch.autograd.Function):
    """u = DDG-PCG(A(exp(theta)), f) with an adjoint backward."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, f: torch.Tensor, ds: DiffusionSolver, refactor: bool = True):
        theta = theta.detach().contiguous()
        if refactor:
            ds.refactor(theta)
        else:
            ds.ensure(theta)
        u = ds.solve(f.detach().contiguous())
        ctx.ds = ds
        ctx.save_for_backward(theta, u)
        return u

    @staticmethod
    def backward(ctx, grad_u: torch.Tensor):
        theta, u = ctx.saved_tensors
        ds = ctx.ds
        # another forward may have refactored the shared handle since this one ran
        ds.ensure(theta)
        lam = ds.solve(grad_u.contiguous())
        grad_theta = ds.coeff_grad(theta, u, lam)
        return grad_theta, lam, None, None


def ddg_solve_fn(theta: torch.Tensor, f: torch.Tensor, ds: DiffusionSolver, refactor: bool = True):
    return DDGSolveFunction.apply(theta, f, ds, refactor)
