"""Shared helpers for the oracle pin tests (CPU only)."""
import itertools

import numpy as np

from oracle.lattice import all_sites


def momenta(dims, antiperiodic_t):
    """All lattice momenta (p_x, p_y, p_z, p_t): 2 pi k / N, or pi (2k+1)/N_t when antiperiodic in t."""
    axes = []
    for mu, n in enumerate(dims):
        if mu == 3 and antiperiodic_t:
            axes.append([np.pi * (2 * k + 1) / n for k in range(n)])
        else:
            axes.append([2 * np.pi * k / n for k in range(n)])
    return [np.array(p) for p in itertools.product(*axes)]


def plane_wave(dims, p, inner):
    """Field exp(i p.n) * inner, indexed [t,z,y,x,...]."""
    nx, ny, nz, nt = dims
    coords = all_sites(dims)
    ph = np.exp(1j * coords @ p).reshape(nt, nz, ny, nx)
    return ph.reshape(ph.shape + (1,) * inner.ndim) * inner


def gauge_rotate_links(U, g):
    """U^g_mu(n) = g(n) U_mu(n) g(n+mu)^dagger (periodic)."""
    out = np.empty_like(U)
    for mu in range(4):
        axis = 3 - mu
        gp = np.roll(g, -1, axis=axis)
        out[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(gp, -1, -2))
    return out


def gauge_rotate_wilson_vector(g, psi):
    """(G psi)(n) = g(n) psi(n) on a (..., Nc, 4, Nv) field."""
    return np.einsum("tzyxab,tzyxbsr->tzyxasr", g, psi)


def gauge_rotate_staggered_vector(g, phi):
    return np.einsum("tzyxab,tzyxbr->tzyxar", g, phi)


def flip_t_boundary(U):
    """Negate the t-links that cross the t boundary (t = Nt-1): periodic twin of the antiperiodic BC."""
    out = U.copy()
    out[-1, :, :, :, 3] *= -1
    return out


def rel_err(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def assert_same_spectrum(ev, expect, atol=1e-10):
    """Multisets of complex eigenvalues agree (optimal one-to-one matching)."""
    from scipy.optimize import linear_sum_assignment

    assert len(ev) == len(expect)
    cost = np.abs(ev[:, None] - expect[None, :])
    r, c = linear_sum_assignment(cost)
    assert np.max(cost[r, c]) < atol, np.max(cost[r, c])
