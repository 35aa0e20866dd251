"""Susskind (staggered) Dirac operator D_S (Sec. 7, Eq. def_stag).

(D_S phi)(n) = m phi(n) + 1/2 sum_mu eta_mu(n) [U_mu(n) b phi(n + mu) - U_mu(n - mu)^dagger b phi(n - mu)]

with eta_1 = 1, eta_2 = (-1)^x, eta_3 = (-1)^(x+y), eta_4 = (-1)^(x+y+z) on
0-based coordinates, and b the fermion boundary sign of the hop.

The adjoint follows from D^dagger(n, m) = D(m, n)^dagger and eta_mu(n + mu) = eta_mu(n):
(D_S^dagger phi)(n) = m phi(n) - 1/2 sum_mu eta_mu(n) [U_mu(n) b phi(n + mu) - U_mu(n - mu)^dagger b phi(n - mu)].
"""
from __future__ import annotations

import numpy as np

from .lattice import all_sites, bc_sign, dims_of_gauge, eta, flat_index, rows, site_field, unit


def _hop(U, phi, coords, dims, antiperiodic_t):
    us = site_field(U)
    ps = site_field(phi)
    n = flat_index(coords, dims)
    h = np.zeros((coords.shape[0],) + ps.shape[1:], dtype=np.complex128)
    for mu in range(4):
        e = unit(mu)
        fwd = flat_index(coords + e, dims)
        bwd = flat_index(coords - e, dims)
        bf = bc_sign(coords, e, dims, antiperiodic_t)[:, None, None]
        bb = bc_sign(coords, -e, dims, antiperiodic_t)[:, None, None]
        up = np.einsum("kab,kbr->kar", rows(us, (n, mu)), rows(ps, fwd)) * bf
        dn = np.einsum("kba,kbr->kar", np.conj(rows(us, (bwd, mu))), rows(ps, bwd)) * bb
        h = h + 0.5 * eta(coords, mu)[:, None, None] * (up - dn)
    return h


def staggered_apply(U, phi, mass, antiperiodic_t=True, sites=None):
    """v = D_S phi.  U: (Nt,Nz,Ny,Nx,4,Nc,Nc); phi: (Nt,Nz,Ny,Nx,Nc,Nv)."""
    dims = dims_of_gauge(U)
    coords = all_sites(dims) if sites is None else np.asarray(sites)
    ps = site_field(phi)
    out = mass * rows(ps, flat_index(coords, dims)) + _hop(U, phi, coords, dims, antiperiodic_t)
    return out.reshape(phi.shape) if sites is None else out


def staggered_apply_dagger(U, phi, mass, antiperiodic_t=True, sites=None):
    """v = D_S^dagger phi = m phi - (hopping part)."""
    dims = dims_of_gauge(U)
    coords = all_sites(dims) if sites is None else np.asarray(sites)
    ps = site_field(phi)
    out = mass * rows(ps, flat_index(coords, dims)) - _hop(U, phi, coords, dims, antiperiodic_t)
    return out.reshape(phi.shape) if sites is None else out
