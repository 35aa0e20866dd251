"""Pins for the Laplace oracle (Eqs. def_wlap/app_wlap and def_blap/app_blap).

* the stencils against dense matrices assembled from the operator-level definitions of Delta^std and
  Delta^bri (the Kronecker-sum builders of ``oracle.dense``), both boundary conditions, several N_c;
* the scalar part of the Dirac operators: -Delta/2 + m^2/2 = (D(m') + D(m')^dagger)/2 with
  m' = m^2/2, for Wilson and Brillouin (the derivative parts are anti-hermitian, Secs. 5 and 6);
* free-field plane-wave eigenvalues in closed form;
* hermiticity, positivity (smallest eigenvalue >= m^2/2 for unitary links), gauge covariance;
* colour-only vectors give the same result as each spin component of a Wilson-layout vector.
"""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle.brillouin import brillouin_apply, brillouin_apply_dagger, brillouin_links, brillouin_links_all
from oracle.dense import _bri_hops, _std_hops
from oracle.gamma import IDENTITY4
from oracle.laplace import (brillouin_laplace_apply, free_brillouin_laplace_symbol, free_wilson_laplace_symbol,
                            wilson_laplace_apply)
from oracle.lattice import dims_of_gauge
from oracle.wilson import wilson_apply, wilson_apply_dagger
from tests.oracle_helpers import gauge_rotate_links, gauge_rotate_wilson_vector, momenta, plane_wave


def _cols(psi):
    return psi.reshape(-1, psi.shape[-1])


def _dense_wlap(U, mass, apbc):
    _, lap = _std_hops(U, apbc)
    n = lap.shape[0] * 4
    return 0.5 * mass * mass * np.eye(n) - 0.5 * np.kron(lap, IDENTITY4)


def _dense_blap(V, mass, apbc):
    dims = dims_of_gauge(V)
    _, lap = _bri_hops(brillouin_links_all(V), dims, apbc)
    n = lap.shape[0] * 4
    return 0.5 * mass * mass * np.eye(n) - 0.5 * np.kron(lap, IDENTITY4)


@pytest.mark.parametrize("dims,nc,apbc", [((2, 2, 2, 2), 2, True), ((2, 2, 2, 4), 3, False),
                                          ((4, 2, 2, 4), 1, True)])
def test_wilson_laplace_equals_dense_definition(dims, nc, apbc):
    rng = np.random.default_rng(21)
    U = si.gauge_field(rng, dims, nc, "haar")
    psi = si.wilson_vector(rng, dims, nc, 2)
    d = _dense_wlap(U, 0.3, apbc)
    np.testing.assert_allclose(_cols(wilson_laplace_apply(U, psi, 0.3, apbc)), d @ _cols(psi), atol=1e-12)
    np.testing.assert_allclose(d, d.conj().T, atol=1e-14)
    assert np.min(np.linalg.eigvalsh(d)) >= 0.5 * 0.3 ** 2 - 1e-12


@pytest.mark.parametrize("dims,nc,apbc", [((2, 2, 2, 2), 2, True), ((2, 2, 2, 4), 2, False)])
def test_brillouin_laplace_equals_dense_definition(dims, nc, apbc):
    rng = np.random.default_rng(22)
    V = si.gauge_field(rng, dims, nc, "haar")
    W = brillouin_links(V)
    psi = si.wilson_vector(rng, dims, nc, 2)
    d = _dense_blap(V, 0.2, apbc)
    np.testing.assert_allclose(_cols(brillouin_laplace_apply(W, psi, 0.2, apbc)), d @ _cols(psi), atol=1e-12)
    np.testing.assert_allclose(d, d.conj().T, atol=1e-14)
    assert np.min(np.linalg.eigvalsh(d)) >= 0.5 * 0.2 ** 2 - 1e-12


def test_laplacians_are_the_scalar_part_of_the_dirac_operators():
    dims, nc, m = (2, 4, 2, 4), 3, 0.4
    rng = np.random.default_rng(23)
    U = si.gauge_field(rng, dims, nc, "near", 0.5)
    psi = si.wilson_vector(rng, dims, nc, 2)
    mp = 0.5 * m * m
    want = 0.5 * (wilson_apply(U, psi, mp) + wilson_apply_dagger(U, psi, mp))
    np.testing.assert_allclose(wilson_laplace_apply(U, psi, m), want, atol=1e-12)
    W = brillouin_links(U)
    want = 0.5 * (brillouin_apply(W, psi, mp) + brillouin_apply_dagger(W, psi, mp))
    np.testing.assert_allclose(brillouin_laplace_apply(W, psi, m), want, atol=1e-12)


@pytest.mark.parametrize("apbc", [True, False])
def test_free_field_plane_waves(apbc):
    dims, nc, m = (4, 2, 2, 4), 2, 0.3
    U = si.gauge_field(None, dims, nc, "unit")
    W = brillouin_links(U)
    rng = np.random.default_rng(24)
    for p in momenta(dims, apbc)[::3]:
        chi = si.complex_gaussian(rng, (nc, 4, 1))
        psi = plane_wave(dims, p, chi)
        np.testing.assert_allclose(wilson_laplace_apply(U, psi, m, apbc), free_wilson_laplace_symbol(p, m) * psi,
                                   atol=1e-13)
        np.testing.assert_allclose(brillouin_laplace_apply(W, psi, m, apbc),
                                   free_brillouin_laplace_symbol(p, m) * psi, atol=1e-13)


def test_gauge_covariance_and_colour_only_vectors():
    dims, nc, m = (2, 2, 2, 4), 3, 0.1
    rng = np.random.default_rng(25)
    U = si.gauge_field(rng, dims, nc, "haar")
    psi = si.wilson_vector(rng, dims, nc, 2)
    g = si.gauge_transform(rng, dims, nc)
    Ug = gauge_rotate_links(U, g)
    for fn, links, links_g in ((wilson_laplace_apply, U, Ug),
                               (brillouin_laplace_apply, brillouin_links(U), brillouin_links(Ug))):
        lhs = fn(links_g, gauge_rotate_wilson_vector(g, psi), m)
        np.testing.assert_allclose(lhs, gauge_rotate_wilson_vector(g, fn(links, psi, m)), atol=1e-12)
        full = fn(links, psi, m)
        for s in range(4):
            np.testing.assert_allclose(fn(links, np.ascontiguousarray(psi[..., s, :]), m), full[..., s, :],
                                       atol=1e-13)
