"""Differentiable GMRES-SDR solve.

``SDRSolve.apply(values, b, solver, tol, adj_tol)`` returns x with
A(values) x = b, where ``values`` are the stored CSR entries of A on the
solver's fixed pattern.  The backward pass runs an adjoint GMRES-SDR solve
A^T lam = dL/dx (A^H for complex data) in the library, whose recycle space is
kept across calls (so successive optimisation steps recycle), and then forms

    dL/dA_e = -lam[row(e)] * x[col(e)]        (complex: -lam * conj(x)),
    dL/db   = lam,

on the sparsity pattern with the library's gradient kernel.  Everything is
computed by the HIP library; torch only carries the tensors and the graph.
"""

from __future__ import annotations

import torch


class SDRSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, b, solver, tol=1e-10, adj_tol=None):
        vals = values.detach().contiguous()
        solver.update_matrix(vals)
        x, st = solver.solve(b.detach().contiguous(), tol=tol)
        if not st["converged"]:
            raise RuntimeError(f"forward GMRES-SDR solve did not converge: {st}")
        solver.last_forward_stats = st
        ctx.solver = solver
        ctx.generation = solver.generation
        ctx.adj_tol = tol if adj_tol is None else adj_tol
        ctx.forward_stats = st
        ctx.save_for_backward(x, vals)
        return x

    @staticmethod
    def backward(ctx, gx):
        x, vals = ctx.saved_tensors
        if ctx.solver.generation != ctx.generation:
            # the shared solver was given another matrix since this node's
            # forward (a second forward before backward): restore this one's
            ctx.solver.update_matrix(vals)
        lam, st = ctx.solver.solve_adjoint(gx.contiguous(), tol=ctx.adj_tol)
        if not st["converged"]:
            raise RuntimeError(f"adjoint GMRES-SDR solve did not converge: {st}")
        ctx.solver.last_adjoint_stats = st
        gvals = ctx.solver.grad_values(lam, x)
        return gvals, lam, None, None, None


def sdr_solve(values, b, solver, tol=1e-10, adj_tol=None):
    """Functional form of :class:`SDRSolve`."""
    return SDRSolve.apply(values, b, solver, tol, adj_tol)
