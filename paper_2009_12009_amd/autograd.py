"""Differentiable solve: phi = A(b)^{-1} f with b = exp(log b) on faces.

The backward pass reuses the same solver handle for the adjoint solve
lambda = A^{-1} g_phi (A is symmetric), returns dL/df = lambda and calls the
library's face-gradient kernel for dL/dlog b_f = -b_f lambda^T (dA/db_f) phi.

Tensor conventions: f and phi are ghost-free MultiFab data (flat, the solver's
boxes, x fastest per box); log b is three x-fastest global face tensors of
shapes MLMG.global_face_shape(d), one value per physical face.
"""

import torch

from .multifab import MultiFab


class MGSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, logb_x, logb_y, logb_z, solver, rel_tol=1e-10, abs_tol=0.0,
                warm_start=None):
        logb = [t.detach().contiguous() for t in (logb_x, logb_y, logb_z)]
        solver.set_coefficients_global(logb, is_log=True)
        rhs = MultiFab(solver.boxes, 0, data=f.detach().contiguous())
        phi = solver.cell_mf(1, fill=0.0)
        if warm_start is not None:
            solver.copy_valid(MultiFab(solver.boxes, 0, data=warm_start.detach().contiguous()), phi)
        solver.solve(phi, rhs, rel_tol, abs_tol)
        out = solver.cell_mf(0)
        solver.copy_valid(phi, out)
        ctx.solver = solver
        ctx.phi = phi
        ctx.tol = (rel_tol, abs_tol)
        ctx.version = solver.coef_version
        ctx.logb = logb
        return out.data

    @staticmethod
    def backward(ctx, g_phi):
        solver = ctx.solver
        if solver.coef_version != ctx.version:
            solver.set_coefficients_global(ctx.logb, is_log=True)
        rhs = MultiFab(solver.boxes, 0, data=g_phi.detach().contiguous())
        lam = solver.cell_mf(1, fill=0.0)
        solver.solve(lam, rhs, *ctx.tol)
        grad_f = solver.cell_mf(0)
        solver.copy_valid(lam, grad_f)
        gx, gy, gz = solver.face_grad_logb_global(ctx.phi, lam)
        return grad_f.data, gx, gy, gz, None, None, None, None


def mg_solve(f, logb_x, logb_y, logb_z, solver, rel_tol=1e-10, abs_tol=0.0, warm_start=None):
    return MGSolve.apply(f, logb_x, logb_y, logb_z, solver, rel_tol, abs_tol, warm_start)
