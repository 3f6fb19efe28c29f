"""Differentiable RSD solves: x = K(theta)^{-1} b as a torch.autograd.Function.

K(theta) = sum_e k(theta_e) K_e (include/rsd_fe.h: k = theta or exp(theta)) is
assembled on the device by rsd_fe_assemble and set up by rsd_setup /
rsd_update_values; the forward solve is rsd_solve (RSD-preconditioned FGMRES).
The backward pass is the adjoint method: differentiating K x = b gives, for a loss
L(x), lambda = K^{-T} dL/dx, dL/db = lambda and dL/dtheta_e = -k'(theta_e)
lambda_e^T K_e x_e.  K is symmetric, so lambda comes from rsd_solve with the same
handle and right-hand side dL/dx; the element sums run in rsd_fe_grad.  This module
only marshals arguments: every step runs in librsd.so.
"""
from __future__ import annotations

import numpy as np
import torch

from .rsd import RSD, FEMap, RSDError, rsd_fe_assemble, rsd_fe_grad


class DifferentiableSolve:
    """Holds the structure, the coefficient map and one RSD handle.

    Calling ``solver(theta, b)`` returns x = K(theta)^{-1} b and records the solve for
    autograd (theta: E float64, b: n float64, both on the device).
    """

    def __init__(self, row_ptr, col_idx, parent, dof_node, fe: dict, kind: str = "exp",
                 rtol: float = 1e-10, restart: int = 30, maxit: int = 1000, **precision):
        dev = torch.device("cuda", torch.cuda.current_device())
        self.row_ptr = torch.as_tensor(np.ascontiguousarray(row_ptr, dtype=np.int64), device=dev)
        self.col_idx = torch.as_tensor(np.ascontiguousarray(col_idx, dtype=np.int32), device=dev)
        self.parent = torch.as_tensor(np.ascontiguousarray(parent, dtype=np.int32), device=dev)
        self.dof_node = torch.as_tensor(np.ascontiguousarray(dof_node, dtype=np.int32), device=dev)
        self.map = FEMap(fe, dev)
        self.kind = kind
        self.values = torch.empty(self.map.nnz, dtype=torch.float64, device=dev)
        self.n = self.row_ptr.numel() - 1
        self.solve_kw = dict(rtol=rtol, restart=restart, maxit=maxit)
        self.precision = precision
        self.rsd = None
        self._theta = None
        self.last_info = []

    def factor(self, theta: torch.Tensor):
        """Assembles K(theta) and sets up (or refreshes) the preconditioner."""
        if self._theta is not None and torch.equal(self._theta, theta):
            return
        rsd_fe_assemble(self.map, theta, self.kind, self.values)
        if self.rsd is None:
            self.rsd = RSD(self.row_ptr, self.col_idx, self.values, self.parent, self.dof_node,
                           **self.precision)
        else:
            self.rsd.update_values(self.values)
        self._theta = theta.detach().clone()

    def solve(self, rhs: torch.Tensor) -> torch.Tensor:
        x, st, info = self.rsd.solve(rhs.contiguous(), **self.solve_kw)
        self.last_info.append(info[0])
        if st != 0:
            raise RSDError(st, f"solve failed: {info[0]}")
        return x

    def __call__(self, theta: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
        return _RSDSolve.apply(theta, b, self)

    def close(self):
        if self.rsd is not None:
            self.rsd.close()
            self.rsd = None
        self._theta = None


class _RSDSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, b, system: DifferentiableSolve):
        theta = theta.detach().contiguous()
        system.factor(theta)
        x = system.solve(b.detach())
        ctx.system = system
        ctx.save_for_backward(theta, x)
        return x

    @staticmethod
    def backward(ctx, gx):
        theta, x = ctx.saved_tensors
        system = ctx.system
        system.factor(theta)                 # refactors only if another forward moved K
        lam = system.solve(gx.detach())      # K symmetric: the adjoint operator is K
        g_theta = torch.empty_like(theta)
        rsd_fe_grad(system.map, theta, system.kind, lam, x, g_theta)
        return g_theta, lam, None
