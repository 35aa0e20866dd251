"""Krylov solvers on multi-RHS fields (Sec. 9), N_v independent solves in lock-step.

Vectors are fields whose last axis is the right-hand-side index; inner
products <u, v> = sum conj(u) v are linear in the second argument (Sec. 3) and
are taken per RHS over every other axis.

Stopping and recompute rules (Sec. 9): the residual r = b - A x is recomputed
explicitly (instead of using the updated one) when (i) the iteration count is
a multiple of ``recompute_every`` (20 in single, 50 in double precision),
(ii) the updated residual suggests ||r|| < tol ||b|| for every RHS, or (iii)
the iteration limit is reached.  The solve ends when the recomputed residual
meets the tolerance for every RHS, when updated and recomputed residual norms
differ by more than 1 %, or at the iteration limit.  A RHS whose recomputed
residual meets the tolerance is frozen (its step lengths are set to zero); the
paper does not say how converged columns are treated inside a multi-RHS solve.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def dot(u, v):
    """Per-RHS <u, v> = sum conj(u) v over all axes but the last."""
    return np.sum((np.conj(u) * v).reshape(-1, u.shape[-1]), axis=0)


def norm2(u):
    return np.sum((np.abs(u) ** 2).reshape(-1, u.shape[-1]), axis=0)


@dataclass
class SolveResult:
    x: np.ndarray
    status: str  # "converged", "stagnated", "maxit"
    iterations: int
    true_relres: np.ndarray
    alphas: list = field(default_factory=list)
    betas: list = field(default_factory=list)


def cg(apply_a, b, x0=None, tol=1e-10, maxit=1000, recompute_every=50, drift=0.01):
    """Conjugate gradients (Hestenes-Stiefel) for hermitian positive definite A, per RHS."""
    x = np.zeros_like(b) if x0 is None else x0.astype(b.dtype, copy=True)
    bnorm = np.sqrt(norm2(b))
    goal = tol * bnorm
    r = b - apply_a(x)
    rr = norm2(r)
    active = np.sqrt(rr) > goal
    p = r.copy()
    alphas, betas = [], []
    status, it = "converged", 0
    while np.any(active):
        if it >= maxit:
            status = "maxit"
            break
        it += 1
        q = apply_a(p)
        pq = dot(p, q).real
        ok = active & (pq > 0)
        alpha = np.where(ok, rr / np.where(ok, pq, 1.0), 0.0)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = norm2(r)
        alphas.append(alpha.copy())
        if it % recompute_every == 0 or np.all(np.sqrt(rr_new[active]) <= goal[active]) or it == maxit:
            r_true = b - apply_a(x)
            rt = norm2(r_true)
            gap = np.abs(np.sqrt(rr_new) - np.sqrt(rt)) / np.maximum(np.sqrt(rt), 1e-300)
            r, rr_new = r_true, rt
            still = active & (np.sqrt(rt) > goal)
            if np.any(still & (gap > drift)):
                active = still
                status = "stagnated"
                break
            active = still
        beta = np.where(active, rr_new / np.where(rr > 0, rr, 1.0), 0.0)
        betas.append(beta.copy())
        p = r + beta * p
        rr = rr_new
    if np.any(active) and status == "converged":
        status = "maxit"
    true_rel = np.sqrt(norm2(b - apply_a(x))) / np.where(bnorm > 0, bnorm, 1.0)
    return SolveResult(x, status, it, true_rel, alphas, betas)


def bicgstab(apply_d, b, x0=None, tol=1e-10, maxit=1000, recompute_every=50, drift=0.01):
    """BiCGstab (van der Vorst 1992) for general D, per RHS, shadow residual r_hat = r_0.

    On breakdown (|rho| or |<r_hat, v>| below 1e-30 ||r_hat|| ||r||, or omega = 0) the
    affected RHS restarts with r_hat = r.  Recompute/exit rules as for ``cg``.
    """
    x = np.zeros_like(b) if x0 is None else x0.astype(b.dtype, copy=True)
    bnorm = np.sqrt(norm2(b))
    goal = tol * bnorm
    r = b - apply_d(x)
    rhat = r.copy()
    nv = b.shape[-1]
    rho = np.ones(nv, dtype=np.complex128)
    alpha = np.ones(nv, dtype=np.complex128)
    omega = np.ones(nv, dtype=np.complex128)
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    active = np.sqrt(norm2(r)) > goal
    status, it = "converged", 0
    while np.any(active):
        if it >= maxit:
            status = "maxit"
            break
        it += 1
        rho_new = dot(rhat, r)
        tiny = 1e-30 * np.sqrt(norm2(rhat) * norm2(r))
        restart = active & ((np.abs(rho_new) <= tiny) | (np.abs(omega) == 0))
        if np.any(restart):
            rhat = np.where(restart, r, rhat)
            rho_new = np.where(restart, norm2(r).astype(np.complex128), rho_new)
            p = np.where(restart, 0.0, p)
            v = np.where(restart, 0.0, v)
            rho = np.where(restart, 1.0, rho)
            alpha = np.where(restart, 1.0, alpha)
            omega = np.where(restart, 1.0, omega)
        beta = np.where(active, (rho_new / rho) * (alpha / omega), 0.0)
        p = r + beta * (p - omega * v)
        v = apply_d(p)
        rv = dot(rhat, v)
        good = active & (np.abs(rv) > 1e-30 * np.sqrt(norm2(rhat) * norm2(v)))
        alpha = np.where(good, rho_new / np.where(good, rv, 1.0), 0.0)
        s = r - alpha * v
        t = apply_d(s)
        tt = norm2(t)
        okw = good & (tt > 0)
        omega = np.where(okw, dot(t, s) / np.where(okw, tt, 1.0), 0.0)
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho = np.where(active, rho_new, rho)
        rr = norm2(r)
        if it % recompute_every == 0 or np.all(np.sqrt(rr[active]) <= goal[active]) or it == maxit:
            r_true = b - apply_d(x)
            rt = norm2(r_true)
            gap = np.abs(np.sqrt(rr) - np.sqrt(rt)) / np.maximum(np.sqrt(rt), 1e-300)
            r = r_true
            still = active & (np.sqrt(rt) > goal)
            if np.any(still & (gap > drift)):
                active = still
                status = "stagnated"
                break
            active = still
    if np.any(active) and status == "converged":
        status = "maxit"
    true_rel = np.sqrt(norm2(b - apply_d(x))) / np.where(bnorm > 0, bnorm, 1.0)
    return SolveResult(x, status, it, true_rel)


def lanczos_extremes(alphas, betas):
    """Extremal eigenvalue estimates of A from one RHS's CG coefficients.

    The CG step lengths alpha_k and ratios beta_k define the Lanczos tridiagonal
    matrix T with diagonal 1/alpha_1, 1/alpha_k + beta_{k-1}/alpha_{k-1} and
    off-diagonal sqrt(beta_k)/alpha_k; its extreme eigenvalues approximate those
    of A (the service of the paper's ``testknl_cond``, App. F).
    """
    a = np.asarray(alphas, dtype=np.float64)
    bt = np.asarray(betas, dtype=np.float64)[: len(a) - 1]
    n = len(a)
    diag = np.empty(n)
    diag[0] = 1.0 / a[0]
    for k in range(1, n):
        diag[k] = 1.0 / a[k] + bt[k - 1] / a[k - 1]
    off = np.sqrt(bt) / a[:-1]
    t = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    ev = np.linalg.eigvalsh(t)
    return ev[0], ev[-1]
