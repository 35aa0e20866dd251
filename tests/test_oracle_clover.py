"""Pins for the clover oracle (Sec. 4, Eq. def_clov; sigma_{mu nu} of App. A).

* F_{mu nu} of a constant abelian field embedded along a traceless Cartan direction T has the closed
  form -sin(theta T) (or +sin(theta T) with the roles of mu and nu exchanged) in its own plane and
  vanishes in the other five: this fixes the 1/8 normalisation, the sense of every leaf, the plane
  order and the periodic wrap.
* sigma_{mu nu} as used by the apply equals the Pauli tensor forms printed in App. A
  (tests/golden/appA_sigma.txt), through a dense per-site matrix built from the printed forms.
* F is traceless hermitian and gauge covariant; C is hermitian, commutes with gamma_5, vanishes in
  the free field and is linear in c_SW.
"""
import os

import numpy as np
import pytest

import synthetic_inputs as si
from oracle.clover import PLANES, clover_apply, clover_site_matrix, field_strength
from oracle.dense import wilson_dense
from oracle.gamma import GAMMA5, PAULI
from oracle.wilson import wilson_apply, wilson_apply_dagger
from tests.oracle_helpers import gauge_rotate_links, gauge_rotate_wilson_vector


def _cartan(nc):
    t = np.zeros(nc)
    t[0], t[1] = 1.0, -1.0
    return t


def _abelian_field(dims, nc, mu, nu, flip):
    """U_mu(n) = exp(i theta n_nu T) (flip: U_nu(n) = exp(i theta n_mu T)), all other links 1;
    theta = 2 pi / N along the coordinate used, so the field is periodic."""
    U = si.gauge_field(None, dims, nc, "unit")
    link, coord = (nu, mu) if flip else (mu, nu)
    theta = 2.0 * np.pi / dims[coord]
    nx, ny, nz, nt = dims
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    c = (x, y, z, t)[coord]
    phase = np.exp(1j * theta * c[..., None] * _cartan(nc))
    U[..., link, :, :] = phase[..., :, None] * np.eye(nc)
    return U, theta


@pytest.mark.parametrize("plane", range(6))
@pytest.mark.parametrize("flip", [False, True])
def test_abelian_field_strength_closed_form(plane, flip):
    dims, nc = (4, 6, 4, 8), 3
    mu, nu = PLANES[plane]
    U, theta = _abelian_field(dims, nc, mu, nu, flip)
    F = field_strength(U)
    expect = (1.0 if flip else -1.0) * np.diag(np.sin(theta * _cartan(nc)))
    for p in range(6):
        want = expect if p == plane else np.zeros((nc, nc))
        np.testing.assert_allclose(F[..., p, :, :], np.broadcast_to(want, F[..., p, :, :].shape), atol=1e-14)


def _printed_sigma(golden_dir):
    sig = {}
    for ln in open(os.path.join(golden_dir, "appA_sigma.txt")):
        if not ln.strip() or ln.startswith("#"):
            continue
        mu, nu, sign, a, b = ln.split()
        sig[(int(mu) - 1, int(nu) - 1)] = float(sign) * np.kron(PAULI[int(a)], PAULI[int(b)])
    return sig


def test_apply_matches_printed_sigma(golden_dir):
    """C psi against the per-site matrix -(c/2) sum F (x) sigma built from the App. A tensor forms."""
    dims, nc, csw = (2, 2, 2, 4), 3, 1.3
    rng = np.random.default_rng(5)
    U = si.gauge_field(rng, dims, nc, "haar")
    psi = si.wilson_vector(rng, dims, nc, 3)
    F = field_strength(U)
    sig = _printed_sigma(golden_dir)
    out = clover_apply(F, psi, csw)
    for t, z, y, x in np.ndindex(dims[3], dims[2], dims[1], dims[0]):
        m = -0.5 * csw * sum(np.kron(F[t, z, y, x, p], sig[PLANES[p]]) for p in range(6))
        v = psi[t, z, y, x].reshape(nc * 4, -1)
        np.testing.assert_allclose(out[t, z, y, x].reshape(nc * 4, -1), m @ v, atol=1e-13)
        np.testing.assert_allclose(clover_site_matrix(F[t, z, y, x], csw), m, atol=1e-14)


def test_field_strength_traceless_hermitian_and_covariant():
    dims, nc = (2, 4, 2, 4), 3
    rng = np.random.default_rng(7)
    U = si.gauge_field(rng, dims, nc, "near", 0.4)
    F = field_strength(U)
    np.testing.assert_allclose(F, np.conj(np.swapaxes(F, -1, -2)), atol=1e-14)
    np.testing.assert_allclose(np.trace(F, axis1=-2, axis2=-1), 0.0, atol=1e-14)
    assert np.max(np.abs(F)) > 1e-2
    g = si.gauge_transform(rng, dims, nc)
    Fg = field_strength(gauge_rotate_links(U, g))
    gd = np.conj(np.swapaxes(g, -1, -2))
    np.testing.assert_allclose(Fg, g[..., None, :, :] @ F @ gd[..., None, :, :], atol=1e-13)


def test_clover_hermitian_chiral_free_and_linear():
    dims, nc = (2, 2, 4, 4), 2
    rng = np.random.default_rng(9)
    U = si.gauge_field(rng, dims, nc, "haar")
    F = field_strength(U)
    g5 = np.kron(np.eye(nc), GAMMA5)
    for site in [(0, 0, 0, 0), (3, 1, 1, 0), (2, 3, 0, 1)]:
        m = clover_site_matrix(F[site], 1.0)
        np.testing.assert_allclose(m, m.conj().T, atol=1e-14)
        np.testing.assert_allclose(m @ g5, g5 @ m, atol=1e-14)
        assert np.max(np.abs(m)) > 1e-3
    psi = si.wilson_vector(rng, dims, nc, 2)
    np.testing.assert_allclose(clover_apply(F, psi, 2.0), 2.0 * clover_apply(F, psi, 1.0), atol=1e-14)
    free = field_strength(si.gauge_field(None, dims, nc, "unit"))
    assert np.max(np.abs(clover_apply(free, psi, 1.0))) == 0.0


def test_clover_improved_operator_adjoint():
    """(D_W + C)^dagger = D_W^dagger + C on the dense matrices (C hermitian, site diagonal)."""
    dims, nc, m, csw = (2, 2, 2, 2), 2, 0.1, 1.0
    rng = np.random.default_rng(13)
    U = si.gauge_field(rng, dims, nc, "haar")
    F = field_strength(U)
    psi = si.wilson_vector(rng, dims, nc, 2)
    cols = psi.reshape(-1, 2)
    d = wilson_dense(U, m, True)
    n = d.shape[0]
    cden = np.zeros((n, n), dtype=np.complex128)
    blk = 4 * nc
    nx, ny, nz, nt = dims
    for t in range(nt):
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    k = ((t * nz + z) * ny + y) * nx + x
                    cden[k * blk:(k + 1) * blk, k * blk:(k + 1) * blk] = clover_site_matrix(F[t, z, y, x], csw)
    full = d + cden
    lhs = (wilson_apply(U, psi, m) + clover_apply(F, psi, csw)).reshape(-1, 2)
    np.testing.assert_allclose(lhs, full @ cols, atol=1e-12)
    lhs = (wilson_apply_dagger(U, psi, m) + clover_apply(F, psi, csw)).reshape(-1, 2)
    np.testing.assert_allclose(lhs, full.conj().T @ cols, atol=1e-12)


def test_clover_gauge_covariant_apply():
    dims, nc, csw = (2, 2, 2, 4), 3, 1.0
    rng = np.random.default_rng(17)
    U = si.gauge_field(rng, dims, nc, "haar")
    psi = si.wilson_vector(rng, dims, nc, 2)
    g = si.gauge_transform(rng, dims, nc)
    lhs = clover_apply(field_strength(gauge_rotate_links(U, g)), gauge_rotate_wilson_vector(g, psi), csw)
    rhs = gauge_rotate_wilson_vector(g, clover_apply(field_strength(U), psi, csw))
    np.testing.assert_allclose(lhs, rhs, atol=1e-13)
