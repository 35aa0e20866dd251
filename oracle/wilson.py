"""Wilson Dirac operator D_W at r = 1, c_SW = 0 (Sec. 5).

(D_W psi)(n) = (4 + m) psi(n)
             + 1/2 sum_mu { [(gamma_mu - 1) x U_mu(n)] b psi(n + mu)
                          - [(gamma_mu + 1) x U_mu(n - mu)^dagger] b psi(n - mu) }

is Eq. app_wils (lattice spacing a = 1); b is the fermion boundary sign of the
hop (see ``lattice.bc_sign``).  The oracle applies the full 4x4 gamma matrices;
it does not use the spin-projection trick of App. A.

The adjoint is written out from D^dagger(n, m) = D(m, n)^dagger:
(D_W^dagger psi)(n) = (4 + m) psi(n)
             - 1/2 sum_mu { [(gamma_mu + 1) x U_mu(n)] b psi(n + mu)
                          - [(gamma_mu - 1) x U_mu(n - mu)^dagger] b psi(n - mu) }.
That it equals gamma_5 D_W gamma_5 (Sec. 9) is checked by the tests, not assumed.
"""
from __future__ import annotations

import numpy as np

from .gamma import GAMMA, IDENTITY4
from .lattice import all_sites, bc_sign, dims_of_gauge, flat_index, rows, site_field, unit


def _hop_terms(U, psi, coords, dims, antiperiodic_t):
    """Yield (mu, U_mu(n) b psi(n+mu), U_mu(n-mu)^dagger b psi(n-mu)) at the given sites."""
    us = site_field(U)
    ps = site_field(psi)
    n = flat_index(coords, dims)
    for mu in range(4):
        e = unit(mu)
        fwd = flat_index(coords + e, dims)
        bwd = flat_index(coords - e, dims)
        bf = bc_sign(coords, e, dims, antiperiodic_t)[:, None, None, None]
        bb = bc_sign(coords, -e, dims, antiperiodic_t)[:, None, None, None]
        up = np.einsum("kab,kbsr->kasr", rows(us, (n, mu)), rows(ps, fwd)) * bf
        # (U^dagger)[a, b] = conj(U[b, a])
        dn = np.einsum("kba,kbsr->kasr", np.conj(rows(us, (bwd, mu))), rows(ps, bwd)) * bb
        yield mu, up, dn


def _spin(mat, f):
    """Act with a 4x4 spin matrix on the spin index of f[k, colour, spin, rhs]."""
    return np.einsum("st,katr->kasr", mat, f)


def _finish(out, psi, sites):
    if sites is None:
        return out.reshape(psi.shape)
    return out


def wilson_apply(U, psi, mass, antiperiodic_t=True, sites=None):
    """v = D_W psi (Eq. app_wils).

    U: (Nt,Nz,Ny,Nx,4,Nc,Nc); psi: (Nt,Nz,Ny,Nx,Nc,4,Nv).  With ``sites`` (an
    (S,4) array of (x,y,z,t)) only those outputs are evaluated, shape (S,Nc,4,Nv).
    """
    dims = dims_of_gauge(U)
    coords = all_sites(dims) if sites is None else np.asarray(sites)
    ps = site_field(psi)
    out = (4.0 + mass) * rows(ps, flat_index(coords, dims))
    for mu, up, dn in _hop_terms(U, psi, coords, dims, antiperiodic_t):
        out = out + 0.5 * _spin(GAMMA[mu] - IDENTITY4, up) - 0.5 * _spin(GAMMA[mu] + IDENTITY4, dn)
    return _finish(out, psi, sites)


def wilson_apply_dagger(U, psi, mass, antiperiodic_t=True, sites=None):
    """v = D_W^dagger psi, the adjoint stencil written out (module docstring)."""
    dims = dims_of_gauge(U)
    coords = all_sites(dims) if sites is None else np.asarray(sites)
    ps = site_field(psi)
    out = (4.0 + mass) * rows(ps, flat_index(coords, dims))
    for mu, up, dn in _hop_terms(U, psi, coords, dims, antiperiodic_t):
        out = out - 0.5 * _spin(GAMMA[mu] + IDENTITY4, up) + 0.5 * _spin(GAMMA[mu] - IDENTITY4, dn)
    return _finish(out, psi, sites)


def free_wilson_symbol(p, mass):
    """Momentum-space D_W at U = 1: m + sum_mu (1 - cos p_mu) + i sum_mu gamma_mu sin p_mu (4x4).

    Follows from Eq. app_wils with psi(n) = exp(i p.n) chi.
    """
    p = np.asarray(p, dtype=np.float64)
    m = (mass + np.sum(1.0 - np.cos(p))) * IDENTITY4
    for mu in range(4):
        m = m + 1j * np.sin(p[mu]) * GAMMA[mu]
    return m
