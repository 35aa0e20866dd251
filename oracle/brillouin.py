"""Brillouin operator D_B at r = 1, c_SW = 0 (Sec. 6) and its hypercube links W.

Directions.  The 81 displacements d = (d_x, d_y, d_z, d_t) in {-1,0,1}^4 are
numbered dir = 27(d_t+1) + 9(d_z+1) + 3(d_y+1) + (d_x+1), so dir = 40 is the
centre (the paper's 1-based "go" loop numbering minus one, App. C).  The 40
directions dir < 40 are stored; the others follow from
W_d(n) = W_{-d}(n+d)^dagger (Tab. off-axis), and -d has number 80 - dir.

Links (Tab. off-axis).  W_d(n) is the plain average, over all |d|! orderings
of the |d| unit steps of d, of the path products V_{s1}(n) V_{s2}(n+s1) ...,
where a step -mu from site x uses V_mu(x - mu)^dagger.  |d| is the number of
non-zero components (1..4 hops; 8, 24, 32, 16 directions with 1, 2, 6, 24 paths).

Operator.  With k = |d|, rho = (64,16,4,1)/432 and lambda = (-240,8,4,2,1)/64,
(D_B psi)(n) = (m - lambda_0/2) psi(n)
             + sum_{d != 0} [(rho_k sum_mu d_mu gamma_mu - lambda_k/2) x W_d(n)] b(n,d) psi(n+d).
This is Eq. app_bril with its shorthand "rho_k gamma_mu" spelled out: the
isotropic derivative of Eq. def_ider puts rho_k W_d(n) into nabla_mu for every
mu with d_mu = +1 and -rho_k W_d(n) for d_mu = -1, so sum_mu gamma_mu nabla_mu
carries rho_k sum_mu d_mu gamma_mu at displacement d.  The dense builder in
``dense`` assembles def_ider/def_blap term by term and the tests compare.

The adjoint D_B^dagger = gamma_5 D_B gamma_5 flips the sign of the rho (derivative)
part: D^dagger(n, n+d) = D(n+d, n)^dagger = (-rho_k sum d_mu gamma_mu - lambda_k/2) x W_d(n).
"""
from __future__ import annotations

import itertools

import numpy as np

from .gamma import GAMMA, IDENTITY4
from .lattice import all_sites, bc_sign, dims_of_gauge, flat_index, rows, site_field, unit

RHO = np.array([0.0, 64.0, 16.0, 4.0, 1.0]) / 432.0  # index k = 1..4 (index 0 unused)
LAMBDA = np.array([-240.0, 8.0, 4.0, 2.0, 1.0]) / 64.0  # index k = 0..4

CENTER = 40
N_STORED = 40


def direction(dir_index: int) -> np.ndarray:
    """Displacement (d_x, d_y, d_z, d_t) of direction number 0..80."""
    dt, r = divmod(dir_index, 27)
    dz, r = divmod(r, 9)
    dy, dx = divmod(r, 3)
    return np.array([dx - 1, dy - 1, dz - 1, dt - 1], dtype=np.int64)


def direction_index(d) -> int:
    return int(27 * (d[3] + 1) + 9 * (d[2] + 1) + 3 * (d[1] + 1) + (d[0] + 1))


def hops(d) -> int:
    return int(np.count_nonzero(d))


def _unit_steps(d):
    return [int(np.sign(d[mu])) * unit(mu) for mu in range(4) if d[mu] != 0]


def _step_link(us, coords, step, dims):
    """Link for one unit step starting at each site: V_mu(x) for +mu, V_mu(x-mu)^dagger for -mu."""
    mu = int(np.flatnonzero(step)[0])
    if step[mu] > 0:
        return rows(us, (flat_index(coords, dims), mu))
    back = rows(us, (flat_index(coords - unit(mu), dims), mu))
    return np.conj(np.swapaxes(back, -1, -2))


def brillouin_links_all(V, sites=None):
    """All 81 W_d(n) at the given sites (default all), shape (S, 81, Nc, Nc); W_centre = 1.

    Each W_d is the average over every ordering of its unit steps of the
    ordered link products along that path (Tab. off-axis).
    """
    dims = dims_of_gauge(V)
    nc = V.shape[-1]
    coords = all_sites(dims) if sites is None else np.asarray(sites)
    us = site_field(V)
    s = coords.shape[0]
    out = np.zeros((s, 81, nc, nc), dtype=np.complex128)
    out[:, CENTER] = np.eye(nc)
    for dir_index in range(81):
        if dir_index == CENTER:
            continue
        d = direction(dir_index)
        steps = _unit_steps(d)
        acc = np.zeros((s, nc, nc), dtype=np.complex128)
        count = 0
        for order in itertools.permutations(range(len(steps))):
            x = coords.copy()
            prod = np.broadcast_to(np.eye(nc, dtype=np.complex128), (s, nc, nc))
            for j in order:
                prod = prod @ _step_link(us, x, steps[j], dims)
                x = x + steps[j]
            acc = acc + prod
            count += 1
        out[:, dir_index] = acc / count
    return out


def brillouin_links(V):
    """Stored links W (Nt,Nz,Ny,Nx,40,Nc,Nc): directions 0..39 of ``brillouin_links_all``."""
    dims = dims_of_gauge(V)
    nx, ny, nz, nt = dims
    nc = V.shape[-1]
    w = brillouin_links_all(V)[:, :N_STORED]
    return w.reshape(nt, nz, ny, nx, N_STORED, nc, nc)


def link_from_stored(W40, coords, dir_index, dims):
    """W_d(n) at the given sites from the 40 stored directions (Tab. off-axis relation)."""
    ws = site_field(W40)
    if dir_index < CENTER:
        return rows(ws, (flat_index(coords, dims), dir_index))
    d = direction(dir_index)
    w = rows(ws, (flat_index(coords + d, dims), 80 - dir_index))
    return np.conj(np.swapaxes(w, -1, -2))


def spin_factor(d, dagger=False) -> np.ndarray:
    """rho_k sum_mu d_mu gamma_mu - lambda_k/2 (4x4) at displacement d != 0; rho part negated for the adjoint."""
    k = hops(d)
    der = sum(d[mu] * GAMMA[mu] for mu in range(4))
    sgn = -1.0 if dagger else 1.0
    return sgn * RHO[k] * der - 0.5 * LAMBDA[k] * IDENTITY4


def _apply_with(link, psi, mass, antiperiodic_t, coords, dims, dagger):
    """D_B (or D_B^dagger) at the given sites; link(dir) returns W_dir at those sites, shape (S, Nc, Nc)."""
    ps = site_field(psi)
    out = (mass - 0.5 * LAMBDA[0]) * rows(ps, flat_index(coords, dims))
    for dir_index in range(81):
        if dir_index == CENTER:
            continue
        d = direction(dir_index)
        w = link(dir_index)
        b = bc_sign(coords, d, dims, antiperiodic_t)[:, None, None, None]
        col = np.einsum("kab,kbsr->kasr", w, rows(ps, flat_index(coords + d, dims))) * b
        out = out + np.einsum("st,katr->kasr", spin_factor(d, dagger), col)
    return out


def _apply(W40, psi, mass, antiperiodic_t, sites, dagger):
    nt, nz, ny, nx = W40.shape[:4]
    dims = (nx, ny, nz, nt)
    coords = all_sites(dims) if sites is None else np.asarray(sites)
    out = _apply_with(lambda k: link_from_stored(W40, coords, k, dims), psi, mass, antiperiodic_t, coords, dims,
                      dagger)
    if sites is None:
        return out.reshape(psi.shape)
    return out


def brillouin_apply(W40, psi, mass, antiperiodic_t=True, sites=None):
    """v = D_B psi (Eq. app_bril with the exact derivative factor); W40 from ``brillouin_links``."""
    return _apply(W40, psi, mass, antiperiodic_t, sites, dagger=False)


def brillouin_apply_dagger(W40, psi, mass, antiperiodic_t=True, sites=None):
    """v = D_B^dagger psi (rho part negated, see module docstring)."""
    return _apply(W40, psi, mass, antiperiodic_t, sites, dagger=True)


def brillouin_apply_sites(W81, psi, mass, sites, antiperiodic_t=True, dagger=False):
    """D_B psi (or D_B^dagger psi) at the given sites from all 81 links there: W81[k, dir] = W_dir(sites[k])
    (as returned by ``brillouin_links_all(V, sites)``).  Avoids the full stored-link array on large lattices."""
    coords = np.asarray(sites)
    nt, nz, ny, nx = psi.shape[:4]
    return _apply_with(lambda k: np.asarray(W81[:, k], dtype=np.complex128), psi, mass, antiperiodic_t, coords,
                       (nx, ny, nz, nt), dagger)


def free_brillouin_symbol(p, mass):
    """Momentum-space D_B at U = 1, summed directly over the 80 displacements (4x4)."""
    p = np.asarray(p, dtype=np.float64)
    m = (mass - 0.5 * LAMBDA[0]) * IDENTITY4
    for dir_index in range(81):
        if dir_index == CENTER:
            continue
        d = direction(dir_index)
        m = m + np.exp(1j * np.dot(p, d)) * spin_factor(d)
    return m
