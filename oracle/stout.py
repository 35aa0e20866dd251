"""Stout smearing of the gauge field (Sec. 2: the smeared links V of the paper's operators; Morningstar
and Peardon's analytic smearing, with the paper's defaults rho = 0.12, three steps).

TEST INFRASTRUCTURE ONLY (see the package docstring).

One step maps U to U' with, for every link,

    C_mu(n)     = rho sum_{nu != mu} [ U_nu(n) U_mu(n+nu) U_nu(n+mu)^+
                                       + U_nu(n-nu)^+ U_mu(n-nu) U_nu(n-nu+mu) ]   (the six staples)
    Omega_mu(n) = C_mu(n) U_mu(n)^+
    Q_mu(n)     = (i/2) (Omega^+ - Omega) - (i/(2 N_c)) Tr(Omega^+ - Omega)       (traceless hermitian)
    U'_mu(n)    = exp(i Q_mu(n)) U_mu(n),

all links updated at once from the old field; n steps repeat this.  The exponential of i Q is taken
through the eigen-decomposition of the hermitian Q.  Links are periodic.
"""
from __future__ import annotations

import numpy as np


def _shift(f, mu, s):
    """g(n) = f(n + s * mu_hat) on a field indexed [t, z, y, x, ...] (periodic)."""
    return np.roll(f, -s, axis=3 - mu)


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def staples(U, mu, rho):
    """C_mu(n) = rho * (sum of the six staples around U_mu(n)), shape (Nt,Nz,Ny,Nx,Nc,Nc)."""
    Um = U[..., mu, :, :]
    c = np.zeros_like(Um)
    for nu in range(4):
        if nu == mu:
            continue
        Un = U[..., nu, :, :]
        c = c + Un @ _shift(Um, nu, 1) @ _dag(_shift(Un, mu, 1))
        Unb = _shift(Un, nu, -1)
        c = c + _dag(Unb) @ _shift(Um, nu, -1) @ _shift(_shift(Un, nu, -1), mu, 1)
    return rho * c


def stout_q(U, rho):
    """Q_mu(n) for every link, shape (Nt,Nz,Ny,Nx,4,Nc,Nc)."""
    nc = U.shape[-1]
    out = np.empty_like(U)
    for mu in range(4):
        om = staples(U, mu, rho) @ _dag(U[..., mu, :, :])
        a = _dag(om) - om
        tr = np.trace(a, axis1=-2, axis2=-1) / nc
        out[..., mu, :, :] = 0.5j * (a - tr[..., None, None] * np.eye(nc))
    return out


def expi_hermitian(q):
    """exp(i Q) for hermitian Q, through its eigen-decomposition."""
    w, v = np.linalg.eigh(q)
    return (v * np.exp(1j * w)[..., None, :]) @ _dag(v)


def stout_step(U, rho):
    """One stout step: U'_mu(n) = exp(i Q_mu(n)) U_mu(n)."""
    return expi_hermitian(stout_q(U, rho)) @ U


def stout_smear(U, rho=0.12, steps=3):
    """``steps`` stout steps with parameter ``rho`` (the paper's defaults)."""
    V = np.array(U, dtype=np.complex128)
    for _ in range(steps):
        V = stout_step(V, rho)
    return V


def mean_plaquette(U):
    """Average of Re Tr(plaquette)/N_c over all sites and the six planes (1 for the free field)."""
    nc = U.shape[-1]
    acc = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Um, Un = U[..., mu, :, :], U[..., nu, :, :]
            p = Um @ _shift(Un, mu, 1) @ _dag(_shift(Um, nu, 1)) @ _dag(Un)
            acc += np.mean(np.trace(p, axis1=-2, axis2=-1).real) / nc
    return acc / 6.0
