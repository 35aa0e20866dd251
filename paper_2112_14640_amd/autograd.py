"""Differentiable front end: torch.autograd.Functions over libdirac.

Gradient convention is torch's for real losses of complex tensors:
grad = dL/dRe + i dL/dIm, so that dL = Re sum conj(grad) * d(tensor).

* ``DiracApply``  v = D(U) u.  Backward: grad_u = D^dagger grad_v (the adjoint apply) and
  grad_U = d Re(grad_v^dagger D(U) u)/dU, the outer-product force of the library.
* ``DiracSolve``  x = (D^dagger D)^{-1} b by CG.  Backward: lambda = (D^dagger D)^{-1} grad_x
  (the normal operator is hermitian, so the adjoint solve is another CG solve),
  grad_b = lambda, grad_U = -[force(D x, lambda) + force(D lambda, x)].
* ``BrillouinLinks``  W = brillouin_links(V) (Tab. off-axis).  Backward: the path-product chain rule
  of the library, grad_V from grad_W.
* ``StoutSmear``  V = n stout steps of U (Sec. 2).  Backward: one library backward step per smearing
  step, in reverse, from the saved intermediate fields.

Link gradients are FP64.  For Wilson and staggered they are with respect to U; for Brillouin with
respect to the stored links W, which ``BrillouinLinks`` and ``StoutSmear`` carry back to V and U, so
U -> V -> W -> D_B is differentiable end to end.  The Laplace operators and the clover term have no
link gradient here (requesting one raises).
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
            if ctx.op not in ("wilson", "staggered", "brillouin"):
                raise NotImplementedError(f"no link gradient for the {ctx.op} operator")
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
            if ctx.op not in ("wilson", "staggered", "brillouin"):
                raise NotImplementedError(f"no link gradient for the {ctx.op} operator")
            dx = dirac.apply(ctx.op, gauge, x, ctx.mass, ctx.apbc)
            dl = dirac.apply(ctx.op, gauge, lam, ctx.mass, ctx.apbc)
            gU = dirac.force(ctx.op, gauge, dx, lam, -1.0, ctx.apbc)
            dirac.force(ctx.op, gauge, dl, x, -1.0, ctx.apbc, out=gU)
        gb = lam if ctx.needs_input_grad[1] else None
        return gU, gb, None, None, None, None, None, None, None


class BrillouinLinks(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V):
        ctx.save_for_backward(V)
        return dirac.brillouin_links(V)

    @staticmethod
    def backward(ctx, gW):
        (V,) = ctx.saved_tensors
        return dirac.brillouin_links_backward(V, gW.contiguous())


class StoutSmear(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, rho, steps):
        fields = [U]
        for _ in range(steps):
            fields.append(dirac.stout_step(fields[-1], rho))
        ctx.rho = rho
        ctx.save_for_backward(*fields[:-1])
        return fields[-1] if steps else U.clone()

    @staticmethod
    def backward(ctx, gV):
        g = gV.contiguous()
        for U in reversed(ctx.saved_tensors):
            g = dirac.stout_backward(U, g, ctx.rho)
        return g, None, None


def brillouin_links(V):
    """Differentiable W = brillouin_links(V) (FP64)."""
    return BrillouinLinks.apply(V)


def stout_smear(U, rho=0.12, steps=3):
    """Differentiable V = ``steps`` stout steps of U (FP64)."""
    return StoutSmear.apply(U, rho, steps)


def apply(op, gauge, u, mass, antiperiodic_t=True):
    """Differentiable v = D(gauge) u."""
    return DiracApply.apply(gauge, u, op, mass, antiperiodic_t)


def solve_normal(op, gauge, b, mass, tol=1e-12, maxit=10000, inner=None, gauge_lo=None, antiperiodic_t=True):
    """Differentiable x = (D^dagger D)^{-1} b."""
    return DiracSolve.apply(gauge, b, op, mass, tol, maxit, inner, gauge_lo, antiperiodic_t)


def su_force(gauge, grad):
    """Project a link gradient onto su(Nc): F with dL/deps = sum tr(H F) for U -> exp(i eps H) U."""
    return dirac.project_su(gauge, grad)
