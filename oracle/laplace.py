"""The embedded Laplace operators -Delta/2 + m^2/2 (Secs. 5 and 6).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Wilson Laplacian (Eq. app_wlap, from the 9-point Delta^std of Eq. def_wlap):
    (-1/2 Delta^std + m^2/2) psi(n) = (4 + m^2/2) psi(n)
                                      - 1/2 sum_mu [U_mu(n) b psi(n+mu) + U_mu(n-mu)^+ b psi(n-mu)]
Brillouin Laplacian (Eq. app_blap, from the 81-point Delta^bri of Eq. def_blap):
    (-1/2 Delta^bri + m^2/2) psi(n) = (m^2/2 - lambda_0/2) psi(n)
                                      - sum_{d != 0} (lambda_|d| / 2) W_d(n) b psi(n+d)
with lambda = (-240, 8, 4, 2, 1)/64.  Both act on the colour index only: the
spin and right-hand-side indices (everything after colour) are carried along
unchanged, so the functions take Wilson-layout vectors (..., Nc, 4, Nv) as the
paper's "embedded" operators do, and colour-only vectors (..., Nc, Nv) alike.
b is the fermion boundary sign of the field (``lattice.bc_sign``); links are
periodic.  Both operators are hermitian and, for unitary links, positive
definite for m != 0 (the tests check this rather than assume it).
"""
from __future__ import annotations

import numpy as np

from .brillouin import CENTER, LAMBDA, direction, hops, link_from_stored
from .lattice import all_sites, bc_sign, dims_of_gauge, flat_index, rows, site_field, unit


def _colour(mat, f):
    """Act with per-site colour matrices mat[k, a, b] on f[k, b, ...]."""
    return np.einsum("kab,kb...->ka...", mat, f)


def _coords(dims, sites):
    return all_sites(dims) if sites is None else np.asarray(sites)


def wilson_laplace_apply(U, psi, mass, antiperiodic_t=True, sites=None):
    """v = (-Delta^std/2 + m^2/2) psi (Eq. app_wlap); psi (Nt,Nz,Ny,Nx,Nc,...)."""
    dims = dims_of_gauge(U)
    coords = _coords(dims, sites)
    us = site_field(U)
    ps = site_field(psi)
    n = flat_index(coords, dims)
    out = (4.0 + 0.5 * mass * mass) * rows(ps, n)
    extra = (1,) * (psi.ndim - 5)
    for mu in range(4):
        e = unit(mu)
        fwd = flat_index(coords + e, dims)
        bwd = flat_index(coords - e, dims)
        bf = bc_sign(coords, e, dims, antiperiodic_t).reshape((-1, 1) + extra)
        bb = bc_sign(coords, -e, dims, antiperiodic_t).reshape((-1, 1) + extra)
        up = _colour(rows(us, (n, mu)), rows(ps, fwd)) * bf
        dn = _colour(np.conj(np.swapaxes(rows(us, (bwd, mu)), -1, -2)), rows(ps, bwd)) * bb
        out = out - 0.5 * (up + dn)
    return out.reshape(psi.shape) if sites is None else out


def brillouin_laplace_apply(W, psi, mass, antiperiodic_t=True, sites=None):
    """v = (-Delta^bri/2 + m^2/2) psi (Eq. app_blap); W the 40 stored links (Nt,Nz,Ny,Nx,40,Nc,Nc)."""
    dims = dims_of_gauge(W)
    coords = _coords(dims, sites)
    ps = site_field(psi)
    n = flat_index(coords, dims)
    out = (0.5 * mass * mass - 0.5 * LAMBDA[0]) * rows(ps, n)
    extra = (1,) * (psi.ndim - 5)
    for dir_index in range(81):
        if dir_index == CENTER:
            continue
        d = direction(dir_index)
        nb = flat_index(coords + d, dims)
        b = bc_sign(coords, d, dims, antiperiodic_t).reshape((-1, 1) + extra)
        w = link_from_stored(W, coords, dir_index, dims)
        out = out - 0.5 * LAMBDA[hops(d)] * _colour(w, rows(ps, nb)) * b
    return out.reshape(psi.shape) if sites is None else out


def free_wilson_laplace_symbol(p, mass):
    """Plane-wave eigenvalue at U = 1: m^2/2 + sum_mu (1 - cos p_mu) (from Eq. app_wlap)."""
    p = np.asarray(p, dtype=np.float64)
    return 0.5 * mass * mass + float(np.sum(1.0 - np.cos(p)))


def free_brillouin_laplace_symbol(p, mass):
    """Plane-wave eigenvalue at W = 1: m^2/2 + 2 (1 - prod_mu cos^2(p_mu/2)).

    From Eq. app_blap: -lambda_0/2 - sum_{d != 0} (lambda_|d|/2) e^{i p.d}.  Since
    lambda_k = 2^(4-k)/64 for k >= 1, and the sum over all d (the d = 0 term is 16) factorises,
    sum_d 2^(4-|d|) e^{i p.d} = prod_mu (2 + 2 cos p_mu) = 256 prod_mu cos^2(p_mu/2), the eigenvalue
    is m^2/2 + 15/8 - (256 prod cos^2 - 16)/128, which is the closed form above.
    """
    p = np.asarray(p, dtype=np.float64)
    return 0.5 * mass * mass + 2.0 * (1.0 - float(np.prod(np.cos(0.5 * p) ** 2)))
