"""Pins for the stout-smearing oracle (Sec. 2; Morningstar and Peardon's analytic smearing).

* One excited link in an otherwise free field has closed-form smeared links: with U_x(n0) = exp(i phi T)
  (T traceless diagonal), the link itself becomes exp(i (phi T - 6 rho sin(phi T))) and every link whose
  staples contain it becomes exp(+-i rho sin(phi T)), the sign fixed by the sense in which the staple runs
  through U_x(n0); all other links stay 1.  This fixes the staple orientations, the factor 1/2 and the
  sign of Q, and rho.
* Smeared links are special unitary; rho = 0 is the identity; smearing is gauge covariant and raises the
  mean plaquette of a rough field; Q is traceless hermitian.
"""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle.stout import mean_plaquette, stout_q, stout_smear, stout_step
from tests.oracle_helpers import gauge_rotate_links


def _at(U, c, mu):
    x, y, z, t = c
    return U[t, z, y, x, mu]


def _expi_diag(v):
    return np.diag(np.exp(1j * v))


@pytest.mark.parametrize("nc", [2, 3])
def test_single_excited_link_closed_form(nc):
    dims, rho, phi = (4, 4, 4, 4), 0.11, 0.7
    T = np.zeros(nc)
    T[0], T[1] = 1.0, -1.0
    U = si.gauge_field(None, dims, nc, "unit")
    n0 = np.array([1, 2, 1, 2])
    x, y, z, t = n0
    U[t, z, y, x, 0] = _expi_diag(phi * T)
    V = stout_step(U, rho)
    ex, ey, et = np.array([1, 0, 0, 0]), np.array([0, 1, 0, 0]), np.array([0, 0, 0, 1])
    s = np.sin(phi * T)
    np.testing.assert_allclose(_at(V, n0, 0), _expi_diag(phi * T - 6 * rho * s), atol=1e-14)
    # staples of U_y at n0 (forward x staple runs along U_x(n0)) and at n0 + x, n0 - y, n0 + x - y
    np.testing.assert_allclose(_at(V, n0, 1), _expi_diag(rho * s), atol=1e-14)
    np.testing.assert_allclose(_at(V, n0 + ex, 1), _expi_diag(-rho * s), atol=1e-14)
    np.testing.assert_allclose(_at(V, n0 - ey, 1), _expi_diag(-rho * s), atol=1e-14)
    np.testing.assert_allclose(_at(V, n0 + ex - ey, 1), _expi_diag(rho * s), atol=1e-14)
    # the parallel links U_x(n0 +- nu) see U_x(n0) in one staple each
    np.testing.assert_allclose(_at(V, n0 + ey, 0), _expi_diag(rho * s), atol=1e-14)
    np.testing.assert_allclose(_at(V, n0 - et, 0), _expi_diag(rho * s), atol=1e-14)
    np.testing.assert_allclose(_at(V, n0 + ex - et, 3), _expi_diag(rho * s), atol=1e-14)
    np.testing.assert_allclose(_at(V, n0 - et, 3), _expi_diag(-rho * s), atol=1e-14)
    np.testing.assert_allclose(_at(V, (n0 + 2 * ey + 2 * et) % 4, 2), np.eye(nc), atol=1e-15)
    # every other link is untouched: count the links that moved
    moved = np.abs(V - U).reshape(-1, 4, nc * nc).max(-1) > 1e-14
    assert moved.sum() == 1 + 3 * 4 + 3 * 2  # the link, 4 transverse links per plane, 2 parallel per plane


def test_special_unitary_identity_and_covariance():
    dims, nc = (2, 4, 2, 4), 3
    rng = np.random.default_rng(31)
    U = si.gauge_field(rng, dims, nc, "haar")
    V = stout_smear(U, 0.12, 3)
    eye = np.eye(nc)
    np.testing.assert_allclose(V @ np.conj(np.swapaxes(V, -1, -2)), np.broadcast_to(eye, V.shape), atol=1e-13)
    np.testing.assert_allclose(np.linalg.det(V), 1.0, atol=1e-13)
    np.testing.assert_allclose(stout_smear(U, 0.0, 2), U, atol=1e-15)
    g = si.gauge_transform(rng, dims, nc)
    np.testing.assert_allclose(stout_smear(gauge_rotate_links(U, g), 0.12, 2),
                               gauge_rotate_links(stout_smear(U, 0.12, 2), g), atol=1e-12)
    q = stout_q(U, 0.12)
    np.testing.assert_allclose(q, np.conj(np.swapaxes(q, -1, -2)), atol=1e-14)
    np.testing.assert_allclose(np.trace(q, axis1=-2, axis2=-1), 0.0, atol=1e-14)


def test_smearing_smooths_a_rough_field():
    dims, nc = (4, 4, 4, 4), 3
    rng = np.random.default_rng(32)
    U = si.gauge_field(rng, dims, nc, "near", 0.8)
    p0 = mean_plaquette(U)
    p1 = mean_plaquette(stout_smear(U, 0.12, 1))
    p3 = mean_plaquette(stout_smear(U, 0.12, 3))
    assert p0 < p1 < p3 < 1.0
    assert mean_plaquette(si.gauge_field(None, dims, nc, "unit")) == pytest.approx(1.0)
