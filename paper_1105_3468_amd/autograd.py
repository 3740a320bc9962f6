"""Differentiable solves on top of libgmg (torch.autograd.Function wrappers).

fv_solve(kappa, B, n, dim, velocity): X = A(kappa)^{-1} B for the cell-centred
FV convection-diffusion matrix of Eq. (pde).  The forward pass assembles
A(kappa) on the GPU, runs the setup and the FGMRES solve; the backward pass
solves the adjoint system A^T Lambda = dL/dX with the transposed two-grid
preconditioner and returns dL/dB = Lambda and
dL/dkappa_c = -sum_r lambda_r^T (dA/dkappa_c) x_r (GPU kernel over the faces).

sparse_solve(rowptr, col, val, B): X = A^{-1} B for a CSR matrix whose values
may require gradients: dL/dval_p = -sum_r lambda_{i(p),r} x_{j(p),r}.

All compute runs in libgmg; these classes only pass tensors through.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gmg


def face_velocities(n: int, dim: int, velocity, device="cuda"):
    """Face-averaged velocity arrays (x, y[, z]) of a workloads velocity field
    (a callable (n, dim) -> list of numpy arrays), as device tensors."""
    if velocity is None:
        shapes = []
        for d in range(dim):
            sh = [n] * dim
            sh[dim - 1 - d] = n + 1
            shapes.append(np.zeros(sh))
        arrs = shapes
    else:
        arrs = velocity(n, dim)
    return [torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device) for a in arrs]


class FVSolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa, B, n, dim, vel, tol, opts):
        rp, ci, va = gmg.fv_assemble(n, dim, kappa.detach(), vel)
        S = gmg.Solver(rp, ci, va, **opts)
        X, res = S.solve(B.detach(), tol=tol)
        if res.status != gmg.OK:
            raise gmg.GmgError(res.status, f"forward solve did not converge: {res.info}")
        ctx.save_for_backward(kappa.detach(), X)
        ctx.S, ctx.n, ctx.dim, ctx.tol = S, n, dim, tol
        ctx.info = res.info
        return X

    @staticmethod
    def backward(ctx, gX):
        kappa, X = ctx.saved_tensors
        Lam, res = ctx.S.solve_adjoint(gX.contiguous(), tol=ctx.tol)
        if res.status != gmg.OK:
            raise gmg.GmgError(res.status, f"adjoint solve did not converge: {res.info}")
        gk = gmg.fv_kappa_grad(ctx.n, ctx.dim, kappa, Lam, X) if ctx.needs_input_grad[0] else None
        gB = Lam if ctx.needs_input_grad[1] else None
        return gk, gB, None, None, None, None, None


def fv_solve(kappa, B, n, dim, vel, tol=1e-10, **opts):
    """Differentiable X = A(kappa)^{-1} B (B of shape (N,) or (N, nrhs)).
    vel: list of face-velocity device tensors (see face_velocities)."""
    return FVSolveFn.apply(kappa, B, n, dim, vel, tol, opts)


class SparseSolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, val, B, rowptr, col, tol, opts):
        S = gmg.Solver(rowptr, col, val.detach(), **opts)
        X, res = S.solve(B.detach(), tol=tol)
        if res.status != gmg.OK:
            raise gmg.GmgError(res.status, f"forward solve did not converge: {res.info}")
        ctx.save_for_backward(X)
        ctx.S, ctx.rowptr, ctx.col, ctx.tol = S, rowptr, col, tol
        return X

    @staticmethod
    def backward(ctx, gX):
        (X,) = ctx.saved_tensors
        Lam, res = ctx.S.solve_adjoint(gX.contiguous(), tol=ctx.tol)
        if res.status != gmg.OK:
            raise gmg.GmgError(res.status, f"adjoint solve did not converge: {res.info}")
        gv = gmg.pattern_grad(ctx.rowptr, ctx.col, Lam, X) if ctx.needs_input_grad[0] else None
        gB = Lam if ctx.needs_input_grad[1] else None
        return gv, gB, None, None, None, None


def sparse_solve(rowptr, col, val, B, tol=1e-10, **opts):
    """Differentiable X = A^{-1} B for A in CSR form with values `val`."""
    return SparseSolveFn.apply(val, B, rowptr, col, tol, opts)
