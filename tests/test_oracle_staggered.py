"""Pins for the staggered oracle: dense definition, anti-hermiticity, epsilon-hermiticity, free field."""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle.dense import staggered_dense
from oracle.lattice import all_sites, epsilon
from oracle.staggered import staggered_apply, staggered_apply_dagger
from tests.oracle_helpers import (flip_t_boundary, gauge_rotate_links, gauge_rotate_staggered_vector, momenta,
                                  plane_wave)


def _cols(phi):
    return phi.reshape(-1, phi.shape[-1])


@pytest.mark.parametrize("dims,nc,apbc", [((2, 2, 2, 2), 3, True), ((4, 4, 4, 4), 3, True),
                                          ((2, 4, 2, 4), 2, False), ((2, 2, 2, 4), 4, True)])
def test_stencil_equals_dense_definition(dims, nc, apbc):
    rng = np.random.default_rng(21)
    U = si.gauge_field(rng, dims, nc, "haar")
    phi = si.staggered_vector(rng, dims, nc, 3)
    d = staggered_dense(U, 0.05, apbc)
    np.testing.assert_allclose(_cols(staggered_apply(U, phi, 0.05, apbc)), d @ _cols(phi), atol=1e-13)
    np.testing.assert_allclose(_cols(staggered_apply_dagger(U, phi, 0.05, apbc)), d.conj().T @ _cols(phi),
                               atol=1e-13)


def test_massless_antihermitian_and_epsilon_hermitian():
    dims, nc = (4, 2, 2, 4), 3
    rng = np.random.default_rng(22)
    U = si.gauge_field(rng, dims, nc, "haar")
    d0 = staggered_dense(U, 0.0, True)
    np.testing.assert_allclose(d0, -d0.conj().T, atol=1e-15)
    d = staggered_dense(U, 0.3, True)
    eps = np.repeat(epsilon(all_sites(dims)), nc)
    np.testing.assert_allclose(d.conj().T, eps[:, None] * d * eps[None, :], atol=1e-15)


@pytest.mark.parametrize("apbc", [True, False])
def test_free_field_normal_operator(apbc):
    # D_S^dag D_S exp(i p.n) = (m^2 + sum sin^2 p_mu) exp(i p.n) at U = 1
    dims, nc, m = (4, 2, 4, 4), 2, 0.1
    U = si.gauge_field(None, dims, nc, "unit")
    rng = np.random.default_rng(23)
    for p in momenta(dims, apbc)[::7]:
        chi = si.complex_gaussian(rng, (nc, 1))
        phi = plane_wave(dims, p, chi)
        out = staggered_apply_dagger(U, staggered_apply(U, phi, m, apbc), m, apbc)
        np.testing.assert_allclose(out, (m * m + np.sum(np.sin(p) ** 2)) * phi, atol=1e-13)


def test_eta_origin_is_a_gauge_transformation():
    # 1-based coordinates negate eta_2 and eta_4; that equals conjugating with G = diag((-1)^(y+t)).
    dims, nc = (2, 4, 2, 4), 2
    rng = np.random.default_rng(24)
    U = si.gauge_field(rng, dims, nc, "haar")
    d0 = staggered_dense(U, 0.2, True)
    flipped = U.copy()
    flipped[..., 1, :, :] *= -1  # negating eta_2 on every y hop ...
    flipped[..., 3, :, :] *= -1  # ... and eta_4 on every t hop
    d1 = staggered_dense(flipped, 0.2, True)
    c = all_sites(dims)
    g = np.repeat(np.where((c[:, 1] + c[:, 3]) % 2 == 0, 1.0, -1.0), nc)
    np.testing.assert_allclose(d1, g[:, None] * d0 * g[None, :], atol=1e-15)


def test_gauge_covariance_and_boundary():
    dims, nc = (2, 4, 2, 4), 3
    rng = np.random.default_rng(25)
    U = si.gauge_field(rng, dims, nc, "haar")
    phi = si.staggered_vector(rng, dims, nc, 2)
    g = si.gauge_transform(rng, dims, nc)
    lhs = staggered_apply(gauge_rotate_links(U, g), gauge_rotate_staggered_vector(g, phi), 0.1)
    rhs = gauge_rotate_staggered_vector(g, staggered_apply(U, phi, 0.1))
    np.testing.assert_allclose(lhs, rhs, atol=1e-13)
    np.testing.assert_allclose(staggered_apply(U, phi, 0.1, True),
                               staggered_apply(flip_t_boundary(U), phi, 0.1, False), atol=1e-14)
