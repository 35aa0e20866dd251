"""Pins for the Wilson oracle: dense definition, free field, gamma5-hermiticity, covariance."""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle.dense import wilson_dense
from oracle.gamma import GAMMA5
from oracle.wilson import free_wilson_symbol, wilson_apply, wilson_apply_dagger
from tests.oracle_helpers import (assert_same_spectrum, flip_t_boundary, gauge_rotate_links, gauge_rotate_wilson_vector, momenta,
                                  plane_wave, rel_err)


def _cols(psi):
    """(Nt,Nz,Ny,Nx,Nc,4,Nv) -> (N, Nv), flattening (site, colour, spin)."""
    return psi.reshape(-1, psi.shape[-1])


@pytest.mark.parametrize("dims,nc,apbc", [((2, 2, 2, 2), 2, True), ((2, 2, 2, 2), 4, False),
                                          ((2, 2, 2, 4), 3, True), ((4, 4, 4, 4), 3, False)])
def test_stencil_equals_dense_definition(dims, nc, apbc):
    rng = np.random.default_rng(11)
    U = si.gauge_field(rng, dims, nc, "haar")
    psi = si.wilson_vector(rng, dims, nc, 2)
    d = wilson_dense(U, 0.13, apbc)
    np.testing.assert_allclose(_cols(wilson_apply(U, psi, 0.13, apbc)), d @ _cols(psi), atol=1e-12)
    np.testing.assert_allclose(_cols(wilson_apply_dagger(U, psi, 0.13, apbc)), d.conj().T @ _cols(psi), atol=1e-12)


def test_dense_4x4_nv1_haar():
    """Wilson 4^4, Nc=3, Nv=1, Haar links, m=0.1, antiperiodic t: Du and D^dagger u vs the 3072^2 matrix."""
    cfg = si.config("wilson_4x4_dense")
    rng = np.random.default_rng(cfg["seed"])
    U = si.gauge_field(rng, cfg["dims"], cfg["nc"], "haar")
    u = si.wilson_vector(rng, cfg["dims"], cfg["nc"], cfg["nv"])
    d = wilson_dense(U, cfg["mass"], True)
    assert d.shape == (3072, 3072)
    assert rel_err(_cols(wilson_apply(U, u, cfg["mass"])), d @ _cols(u)) < 1e-14
    assert rel_err(_cols(wilson_apply_dagger(U, u, cfg["mass"])), d.conj().T @ _cols(u)) < 1e-14


@pytest.mark.parametrize("apbc", [True, False])
def test_free_field_plane_waves(apbc):
    dims, nc, m = (4, 2, 2, 4), 2, 0.07
    U = si.gauge_field(None, dims, nc, "unit")
    rng = np.random.default_rng(3)
    for p in momenta(dims, apbc)[::3]:
        chi = si.complex_gaussian(rng, (nc, 4, 1))
        psi = plane_wave(dims, p, chi)
        expect = plane_wave(dims, p, np.einsum("st,atr->asr", free_wilson_symbol(p, m), chi))
        np.testing.assert_allclose(wilson_apply(U, psi, m, apbc), expect, atol=1e-13)


def test_free_field_spectrum_closed_form():
    dims, nc, m = (2, 2, 4, 4), 1, 0.05
    U = si.gauge_field(None, dims, nc, "unit")
    ev = np.linalg.eigvals(wilson_dense(U, m, True))
    expect = []
    for p in momenta(dims, True):
        re = m + np.sum(1 - np.cos(p))
        im = np.sqrt(np.sum(np.sin(p) ** 2))
        expect += [re + 1j * im] * 2 + [re - 1j * im] * 2
    assert_same_spectrum(ev, np.array(expect))


def test_free_field_extreme_real_part():
    # the free Wilson spectrum reaches Re z = 8 + m at p = (pi,pi,pi,pi) (Sec. 9)
    m = 0.01
    p = np.array([np.pi] * 4)
    np.testing.assert_allclose(np.diag(free_wilson_symbol(p, m)).real, 8 + m)
    np.testing.assert_allclose(free_wilson_symbol(np.zeros(4), m), m * np.eye(4), atol=1e-15)


def test_gamma5_hermiticity():
    dims, nc = (4, 2, 2, 4), 3
    rng = np.random.default_rng(5)
    U = si.gauge_field(rng, dims, nc, "haar")
    psi = si.wilson_vector(rng, dims, nc, 3)
    g5 = lambda f: np.einsum("st,...atr->...asr", GAMMA5, f)
    np.testing.assert_allclose(wilson_apply_dagger(U, psi, 0.2), g5(wilson_apply(U, g5(psi), 0.2)), atol=1e-13)


def test_gauge_covariance():
    dims, nc = (2, 4, 2, 4), 3
    rng = np.random.default_rng(6)
    U = si.gauge_field(rng, dims, nc, "haar")
    psi = si.wilson_vector(rng, dims, nc, 2)
    g = si.gauge_transform(rng, dims, nc)
    lhs = wilson_apply(gauge_rotate_links(U, g), gauge_rotate_wilson_vector(g, psi), 0.3)
    rhs = gauge_rotate_wilson_vector(g, wilson_apply(U, psi, 0.3))
    np.testing.assert_allclose(lhs, rhs, atol=1e-13)


def test_antiperiodic_equals_flipped_links():
    dims, nc = (2, 2, 2, 4), 2
    rng = np.random.default_rng(8)
    U = si.gauge_field(rng, dims, nc, "haar")
    psi = si.wilson_vector(rng, dims, nc, 2)
    np.testing.assert_allclose(wilson_apply(U, psi, 0.1, True), wilson_apply(flip_t_boundary(U), psi, 0.1, False),
                               atol=1e-14)


def test_rhs_columns_independent_and_sampled_sites():
    dims, nc = (4, 2, 2, 4), 3
    rng = np.random.default_rng(9)
    U = si.gauge_field(rng, dims, nc, "near", 0.3)
    psi = si.wilson_vector(rng, dims, nc, 5)
    full = wilson_apply(U, psi, 0.05)
    for r in range(5):
        np.testing.assert_allclose(full[..., r:r + 1], wilson_apply(U, psi[..., r:r + 1], 0.05), atol=1e-14)
    sites = np.array([[0, 0, 0, 0], [3, 1, 1, 3], [1, 0, 1, 2]])
    sub = wilson_apply(U, psi, 0.05, sites=sites)
    for k, (x, y, z, t) in enumerate(sites):
        np.testing.assert_allclose(sub[k], full[t, z, y, x], atol=1e-14)


def test_derivative_antihermitian_laplacian_hermitian():
    # nabla^std is anti-hermitian and Delta^std hermitian (Sec. 5), also with the boundary signs
    from oracle.dense import _std_hops

    dims, nc = (2, 2, 2, 4), 2
    rng = np.random.default_rng(10)
    U = si.gauge_field(rng, dims, nc, "haar")
    nab, lap = _std_hops(U, True)
    for mu in range(4):
        np.testing.assert_allclose(nab[mu], -nab[mu].conj().T, atol=1e-15)
    np.testing.assert_allclose(lap, lap.conj().T, atol=1e-15)
