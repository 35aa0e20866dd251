"""Lattice geometry: site coordinates, neighbour gathers, boundary signs, phases.

Site n = (x, y, z, t) with 0-based coordinates; arrays are indexed
[t, z, y, x, ...] so x is the fastest site index.  Neighbours are taken modulo
the extents (the paper's periodic box, Sec. 2 and App. B).  Fermion fields may
additionally be antiperiodic in t: a hop that leaves [0, Nt-1] in t picks up a
factor -1 on the fetched spinor, while links stay periodic.
"""
from __future__ import annotations

import numpy as np


def dims_of_gauge(u: np.ndarray):
    """(Nx, Ny, Nz, Nt) of a field indexed [t, z, y, x, ...]."""
    nt, nz, ny, nx = u.shape[:4]
    return (nx, ny, nz, nt)


def all_sites(dims) -> np.ndarray:
    """Coordinates (x, y, z, t) of every site, in memory order (x fastest); shape (V, 4)."""
    nx, ny, nz, nt = dims
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel(), t.ravel()], axis=1)


def flat_index(coords: np.ndarray, dims) -> np.ndarray:
    """Linear site index ((t*Nz + z)*Ny + y)*Nx + x of coordinates (..., 4), taken mod the extents."""
    nx, ny, nz, nt = dims
    c = np.mod(coords, np.array([nx, ny, nz, nt]))
    return ((c[..., 3] * nz + c[..., 2]) * ny + c[..., 1]) * nx + c[..., 0]


def site_field(f: np.ndarray) -> np.ndarray:
    """View a field indexed [t,z,y,x,...] as [site, ...]."""
    return f.reshape((-1,) + f.shape[4:])


def rows(field_sites: np.ndarray, index) -> np.ndarray:
    """Rows of a [site, ...] field as complex128, whatever the storage type (all arithmetic is FP64)."""
    return np.asarray(field_sites[index], dtype=np.complex128)


def bc_sign(coords: np.ndarray, disp, dims, antiperiodic_t: bool) -> np.ndarray:
    """Fermion boundary sign b(n, d): -1 iff antiperiodic in t and t + d_t leaves [0, Nt-1]."""
    nt = dims[3]
    s = np.ones(coords.shape[0])
    if antiperiodic_t and disp[3] != 0:
        tt = coords[:, 3] + disp[3]
        s[(tt < 0) | (tt >= nt)] = -1.0
    return s


def unit(mu: int) -> np.ndarray:
    e = np.zeros(4, dtype=np.int64)
    e[mu] = 1
    return e


def eta(coords: np.ndarray, mu: int) -> np.ndarray:
    """Staggered phase eta_mu(n) = (-1)^(sum of the coordinates before mu), 0-based.

    eta_1 = 1, eta_2 = (-1)^x, eta_3 = (-1)^(x+y), eta_4 = (-1)^(x+y+z) (Eq. def_stag).
    """
    s = np.zeros(coords.shape[0], dtype=np.int64)
    for nu in range(mu):
        s = s + coords[:, nu]
    return np.where(s % 2 == 0, 1.0, -1.0)


def epsilon(coords: np.ndarray) -> np.ndarray:
    """Site parity (-1)^(x+y+z+t) (Sec. 3, the staggered analogue of gamma_5)."""
    return np.where(coords.sum(axis=1) % 2 == 0, 1.0, -1.0)
