"""Link gradients of Dirac bilinears ("fermion force").

Gradient convention (the one torch uses for real losses of complex tensors):
for a real L, g = dL/dRe(U) + i dL/dIm(U), so that dL = Re sum tr(g^dagger dU).

Wilson.  From Eq. app_wils, U_mu(n) enters the hop n -> n+mu as
1/2 (gamma_mu - 1) x U_mu(n) b and the hop n+mu -> n as -1/2 (gamma_mu + 1) x U_mu(n)^dagger b.
Differentiating Re psi^dagger D_W chi therefore gives, per link and summed over
spin s and RHS,
    g_mu(n) = -1/2 b sum_s [ ((1 - gamma_mu) psi(n))_s chi_s(n+mu)^dagger
                           + chi_s(n) ((1 + gamma_mu) psi(n+mu))_s^dagger ]     (Nc x Nc).

Staggered.  Likewise from Eq. def_stag,
    g_mu(n) = 1/2 eta_mu(n) b sum [ psi(n) chi(n+mu)^dagger - chi(n) psi(n+mu)^dagger ].

Solves.  For x = A^{-1} phi with A = D^dagger D and L = sum Re phi^dagger A^{-1} phi,
dL = -2 Re (D chi)^dagger dD chi with chi = A^{-1} phi, so grad_U = -2 g(psi = D chi, chi)
and grad_phi = 2 chi.  For a general x = A^{-1} b with upstream gradient gbar,
lambda = A^{-1} gbar, grad_b = lambda, grad_U = -[g(D x, lambda) + g(D lambda, x)].

Projection.  Under U -> exp(i eps H) U with H hermitian traceless,
dL/deps = tr(H F) with F = (i/2)(U g^dagger - g U^dagger) minus its trace / Nc.
"""
from __future__ import annotations

import numpy as np

from .gamma import GAMMA, IDENTITY4
from .lattice import all_sites, bc_sign, dims_of_gauge, eta, flat_index, site_field, unit


def wilson_force(U, psi, chi, antiperiodic_t=True):
    """g = d Re(psi^dagger D_W chi) / dU, shape of U."""
    dims = dims_of_gauge(U)
    coords = all_sites(dims)
    ps = site_field(np.asarray(psi, dtype=np.complex128))
    cs = site_field(np.asarray(chi, dtype=np.complex128))
    g = np.zeros(site_field(U).shape, dtype=np.complex128)
    for mu in range(4):
        e = unit(mu)
        fwd = flat_index(coords + e, dims)
        b = bc_sign(coords, e, dims, antiperiodic_t)[:, None, None]
        pm = np.einsum("st,katr->kasr", IDENTITY4 - GAMMA[mu], ps)
        pp = np.einsum("st,katr->kasr", IDENTITY4 + GAMMA[mu], ps[fwd])
        t1 = np.einsum("kasr,kbsr->kab", pm, np.conj(cs[fwd]))
        t2 = np.einsum("kasr,kbsr->kab", cs, np.conj(pp))
        g[:, mu] = -0.5 * b * (t1 + t2)
    return g.reshape(U.shape)


def staggered_force(U, psi, chi, antiperiodic_t=True):
    """g = d Re(psi^dagger D_S chi) / dU, shape of U."""
    dims = dims_of_gauge(U)
    coords = all_sites(dims)
    ps = site_field(np.asarray(psi, dtype=np.complex128))
    cs = site_field(np.asarray(chi, dtype=np.complex128))
    g = np.zeros(site_field(U).shape, dtype=np.complex128)
    for mu in range(4):
        e = unit(mu)
        fwd = flat_index(coords + e, dims)
        b = bc_sign(coords, e, dims, antiperiodic_t)[:, None, None]
        et = eta(coords, mu)[:, None, None]
        t1 = np.einsum("kar,kbr->kab", ps, np.conj(cs[fwd]))
        t2 = np.einsum("kar,kbr->kab", cs, np.conj(ps[fwd]))
        g[:, mu] = 0.5 * et * b * (t1 - t2)
    return g.reshape(U.shape)


def project_su(U, g):
    """su(Nc) force F = (i/2)(U g^dagger - g U^dagger) - tr/Nc, hermitian traceless."""
    nc = U.shape[-1]
    ugd = U @ np.conj(np.swapaxes(g, -1, -2))
    gud = g @ np.conj(np.swapaxes(U, -1, -2))
    f = 0.5j * (ugd - gud)
    tr = np.trace(f, axis1=-2, axis2=-1) / nc
    return f - tr[..., None, None] * np.eye(nc)
