"""Brute-force dense matrices assembled from the operator-level definitions.

These are a second, independent formulation of each operator, built term by
term from the defining equations (not from the stencil formulas used by
``wilson``, ``brillouin`` and ``staggered``):

* D_W = sum_mu gamma_mu (x) nabla^std_mu - 1/2 Delta^std + m   (Eqs. def_wils, def_sder, def_wlap)
* D_B = sum_mu gamma_mu (x) nabla^iso_mu - 1/2 Delta^bri + m   (Eqs. def_bril, def_ider, def_blap)
* D_S from Eq. def_stag.

Colour-space hopping matrices act on the index (site, colour); the spin
structure enters through Kronecker products with 4x4 matrices, which matches
the vector flattening (site, colour, spin) of a (Nt,Nz,Ny,Nx,Nc,4) field.
Fermion boundary signs b are put into each hopping block.  Loops are plain
Python over sites: small lattices only (2^4, 4^4).
"""
from __future__ import annotations

import numpy as np

from .brillouin import CENTER, LAMBDA, RHO, direction, direction_index, hops
from .gamma import GAMMA, IDENTITY4
from .lattice import all_sites, bc_sign, dims_of_gauge, eta, flat_index, unit


def _add_block(mat, nc, row_site, col_site, block):
    r0, c0 = row_site * nc, col_site * nc
    mat[r0:r0 + nc, c0:c0 + nc] += block


def _std_hops(U, antiperiodic_t):
    """nabla^std_mu (def_sder) and Delta^std (def_wlap) as (V*Nc)^2 colour matrices."""
    dims = dims_of_gauge(U)
    nc = U.shape[-1]
    coords = all_sites(dims)
    v = coords.shape[0]
    nab = np.zeros((4, v * nc, v * nc), dtype=np.complex128)
    lap = np.zeros((v * nc, v * nc), dtype=np.complex128)
    for k in range(v):
        c = coords[k:k + 1]
        for mu in range(4):
            e = unit(mu)
            nf = int(flat_index(c + e, dims)[0])
            nb = int(flat_index(c - e, dims)[0])
            bf = bc_sign(c, e, dims, antiperiodic_t)[0]
            bb = bc_sign(c, -e, dims, antiperiodic_t)[0]
            fwd = U[tuple(c[0][::-1])][mu]
            back_site = tuple(np.mod(c[0] - e, dims)[::-1])
            bwd = np.conj(U[back_site][mu]).T
            _add_block(nab[mu], nc, k, nf, 0.5 * bf * fwd)
            _add_block(nab[mu], nc, k, nb, -0.5 * bb * bwd)
            _add_block(lap, nc, k, nf, bf * fwd)
            _add_block(lap, nc, k, nb, bb * bwd)
        _add_block(lap, nc, k, k, -8.0 * np.eye(nc))
    return nab, lap


def wilson_dense(U, mass, antiperiodic_t=True):
    """Dense D_W, shape (V*Nc*4)^2, index (site, colour, spin)."""
    nab, lap = _std_hops(U, antiperiodic_t)
    n = lap.shape[0] * 4
    d = mass * np.eye(n, dtype=np.complex128) - 0.5 * np.kron(lap, IDENTITY4)
    for mu in range(4):
        d = d + np.kron(nab[mu], GAMMA[mu])
    return d


def _bri_hops(Wall, dims, antiperiodic_t):
    """nabla^iso_mu (def_ider) and Delta^bri (def_blap) from all-direction links Wall (V,81,Nc,Nc)."""
    nc = Wall.shape[-1]
    coords = all_sites(dims)
    v = coords.shape[0]
    nab = np.zeros((4, v * nc, v * nc), dtype=np.complex128)
    lap = np.zeros((v * nc, v * nc), dtype=np.complex128)
    transverse = [np.array(e) for e in np.ndindex(3, 3, 3, 3)]
    for k in range(v):
        c = coords[k:k + 1]
        # Delta^bri: lambda_0 at the centre, lambda_|d| W_d(n) at n+d
        for dir_index in range(81):
            d = direction(dir_index)
            col = int(flat_index(c + d, dims)[0])
            if dir_index == CENTER:
                _add_block(lap, nc, k, col, LAMBDA[0] * np.eye(nc))
                continue
            b = bc_sign(c, d, dims, antiperiodic_t)[0]
            _add_block(lap, nc, k, col, LAMBDA[hops(d)] * b * Wall[k, dir_index])
        # nabla^iso_mu: for every transverse offset e (e_mu = 0, e may be 0) the pair
        # rho_k [W_{mu+e}(n) delta_{n+mu+e} - W_{-mu+e}(n) delta_{n-mu+e}], k = 1 + |e|
        for mu in range(4):
            for e3 in transverse:
                e = e3 - 1
                if e[mu] != 0:
                    continue
                for sgn in (+1, -1):
                    d = e + sgn * unit(mu)
                    kk = hops(d)
                    col = int(flat_index(c + d, dims)[0])
                    b = bc_sign(c, d, dims, antiperiodic_t)[0]
                    _add_block(nab[mu], nc, k, col, sgn * RHO[kk] * b * Wall[k, direction_index(d)])
    return nab, lap


def brillouin_dense(Wall, dims, mass, antiperiodic_t=True):
    """Dense D_B from the 81-direction links at every site (``brillouin_links_all``)."""
    nab, lap = _bri_hops(Wall, dims, antiperiodic_t)
    n = lap.shape[0] * 4
    d = mass * np.eye(n, dtype=np.complex128) - 0.5 * np.kron(lap, IDENTITY4)
    for mu in range(4):
        d = d + np.kron(nab[mu], GAMMA[mu])
    return d


def staggered_dense(U, mass, antiperiodic_t=True):
    """Dense D_S, shape (V*Nc)^2, index (site, colour) (Eq. def_stag)."""
    dims = dims_of_gauge(U)
    nc = U.shape[-1]
    coords = all_sites(dims)
    v = coords.shape[0]
    d = mass * np.eye(v * nc, dtype=np.complex128)
    for k in range(v):
        c = coords[k:k + 1]
        for mu in range(4):
            e = unit(mu)
            et = eta(c, mu)[0]
            nf = int(flat_index(c + e, dims)[0])
            nb = int(flat_index(c - e, dims)[0])
            bf = bc_sign(c, e, dims, antiperiodic_t)[0]
            bb = bc_sign(c, -e, dims, antiperiodic_t)[0]
            fwd = U[tuple(c[0][::-1])][mu]
            bwd = np.conj(U[tuple(np.mod(c[0] - e, dims)[::-1])][mu]).T
            _add_block(d, nc, k, nf, 0.5 * et * bf * fwd)
            _add_block(d, nc, k, nb, -0.5 * et * bb * bwd)
    return d


def field_to_columns(psi):
    """(Nt,Nz,Ny,Nx,...,Nv) field -> (N, Nv) matrix of flattened columns."""
    return psi.reshape(-1, psi.shape[-1])


def columns_to_field(cols, shape):
    return cols.reshape(shape)
