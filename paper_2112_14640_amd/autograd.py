"""Differentiable front end: torch.autograd.Functions over libdirac.

Gradient convention is torch's for real losses of complex tensors:
grad = dL/dRe + i dL/dIm, so that dL = Re sum conj(grad) * d(tensor).

* ``DiracApply``  v = D(U) u.  Backward: grad_u = D^dagger grad_v (the adjoint apply) and
  grad_U = d Re(grad_v^dagger D(U) u)/dU, the outer-product force of the library.
* ``DiracSolve``  x = (D^dagger D)^{-1} b by CG.  Backward: lambda = (D^dagger D)^{-1} grad_x
  (the normal operator is hermitian, so the adjoint solve is another CG solve),
  grad_b = lambda, grad_U = -[force(D x, lambda) + force(D lambda, x)].

Link gradients are available for Wilson and staggered operators in FP64; for
Brillouin only the vector gradient is provided (grad_W is not implemented and
requesting it raises).
"""
from __future__ import annotations

import torch

from . import dirac


class DiracApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gauge, u, op, mass, antiperiodic_t):
        ctx.op, ctx.mass, ctx.apbc = op, mass, antiperiodic_t
        ctx.save_for_backward(gauge, u)
        return dirac.apply(op, gauge, u, mass, antiperiodic_t)

    @staticmethod
    def backward(ctx, gv):
        gauge, u = ctx.saved_tensors
        gv = gv.contiguous()
        gu = gU = None
        if ctx.needs_input_grad[1]:
            gu = dirac.apply_dagger(ctx.op, gauge, gv, ctx.mass, ctx.apbc)
        if ctx.needs_input_grad[0]:
            if ctx.op == "brillouin":
                raise NotImplementedError("the gradient with respect to the Brillouin links W is not implemented")
            gU = dirac.force(ctx.op, gauge, gv, u, 1.0, ctx.apbc)
        return gU, gu, None, None, None


class DiracSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gauge, b, op, mass, tol, maxit, inner, gauge_lo, antiperiodic_t):
        x, info = dirac.cg(op, gauge, b, mass, tol=tol, maxit=maxit, inner=inner, gauge_lo=gauge_lo,
                           antiperiodic_t=antiperiodic_t)
        if info.reason != "converged":
            raise RuntimeError(f"DiracSolve: CG did not converge ({info.reason}, residuals {info.true_relres})")
        ctx.op, ctx.mass, ctx.tol, ctx.maxit, ctx.inner, ctx.apbc = op, mass, tol, maxit, inner, antiperiodic_t
        ctx.save_for_backward(gauge, x, gauge_lo if gauge_lo is not None else torch.empty(0))
        ctx.has_lo = gauge_lo is not None
        return x

    @staticmethod
    def backward(ctx, gx):
        gauge, x, gauge_lo = ctx.saved_tensors
        gauge_lo = gauge_lo if ctx.has_lo else None
        lam, info = dirac.cg(ctx.op, gauge, gx.contiguous(), ctx.mass, tol=ctx.tol, maxit=ctx.maxit, inner=ctx.inner,
                             gauge_lo=gauge_lo, antiperiodic_t=ctx.apbc)
        if info.reason != "converged":
            raise RuntimeError(f"DiracSolve backward: adjoint CG did not converge ({info.reason})")
        gU = None
        if ctx.needs_input_grad[0]:
            if ctx.op == "brillouin":
                raise NotImplementedError("the gradient with respect to the Brillouin links W is not implemented")
            dx = dirac.apply(ctx.op, gauge, x, ctx.mass, ctx.apbc)
            dl = dirac.apply(ctx.op, gauge, lam, ctx.mass, ctx.apbc)
            gU = dirac.force(ctx.op, gauge, dx, lam, -1.0, ctx.apbc)
            dirac.force(ctx.op, gauge, dl, x, -1.0, ctx.apbc, out=gU)
        gb = lam if ctx.needs_input_grad[1] else None
        return gU, gb, None, None, None, None, None, None, None


def apply(op, gauge, u, mass, antiperiodic_t=True):
    """Differentiable v = D(gauge) u."""
    return DiracApply.apply(gauge, u, op, mass, antiperiodic_t)


def solve_normal(op, gauge, b, mass, tol=1e-12, maxit=10000, inner=None, gauge_lo=None, antiperiodic_t=True):
    """Differentiable x = (D^dagger D)^{-1} b."""
    return DiracSolve.apply(gauge, b, op, mass, tol, maxit, inner, gauge_lo, antiperiodic_t)


def su_force(gauge, grad):
    """Project a link gradient onto su(Nc): F with dL/deps = sum tr(H F) for U -> exp(i eps H) U."""
    return dirac.project_su(gauge, grad)
