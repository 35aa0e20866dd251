"""Pins for the link-gradient oracle: brute-force finite differences on tiny lattices."""
import numpy as np

import synthetic_inputs as si
from oracle.dense import staggered_dense, wilson_dense
from oracle.force import project_su, staggered_force, wilson_force
from oracle.wilson import wilson_apply


def _bilinear_fd_gradient(dense_of_u, U, psi, chi):
    """Every real component of dL/dU for L = Re psi^dag D(U) chi by central differences.

    L is linear in (Re U, Im U), so the difference quotient is exact up to rounding.
    """
    g = np.zeros_like(U)
    p = psi.reshape(-1, psi.shape[-1])
    c = chi.reshape(-1, chi.shape[-1])
    h = 1e-3
    for idx in np.ndindex(U.shape):
        for unit in (1.0, 1j):
            up, dn = U.copy(), U.copy()
            up[idx] += h * unit
            dn[idx] -= h * unit
            lp = np.real(np.sum(np.conj(p) * (dense_of_u(up) @ c)))
            ln = np.real(np.sum(np.conj(p) * (dense_of_u(dn) @ c)))
            g[idx] += unit * (lp - ln) / (2 * h)
    return g


def test_wilson_bilinear_gradient_brute_force():
    dims, nc = (2, 2, 2, 2), 2
    rng = np.random.default_rng(41)
    U = si.gauge_field(rng, dims, nc, "haar")
    psi = si.wilson_vector(rng, dims, nc, 2)
    chi = si.wilson_vector(rng, dims, nc, 2)
    g = wilson_force(U, psi, chi, True)
    fd = _bilinear_fd_gradient(lambda u: wilson_dense(u, 0.1, True), U, psi, chi)
    np.testing.assert_allclose(g, fd, atol=1e-10)


def test_staggered_bilinear_gradient_brute_force():
    dims, nc = (2, 2, 2, 4), 2
    rng = np.random.default_rng(42)
    U = si.gauge_field(rng, dims, nc, "haar")
    psi = si.staggered_vector(rng, dims, nc, 2)
    chi = si.staggered_vector(rng, dims, nc, 2)
    g = staggered_force(U, psi, chi, True)
    fd = _bilinear_fd_gradient(lambda u: staggered_dense(u, 0.1, True), U, psi, chi)
    np.testing.assert_allclose(g, fd, atol=1e-10)


def _solve_loss(U, phi, m):
    d = wilson_dense(U, m, True)
    a = d.conj().T @ d
    f = phi.reshape(-1, phi.shape[-1])
    return np.real(np.sum(np.conj(f) * np.linalg.solve(a, f)))


def test_solve_loss_gradients_finite_differences():
    """L = sum_i Re phi_i^dag (D^dag D)^{-1} phi_i: grad_phi = 2 chi, su(N) force vs exp(i eps H) U."""
    dims, nc, m = (2, 2, 2, 4), 3, 0.2
    rng = np.random.default_rng(43)
    U = si.gauge_field(rng, dims, nc, "near", 0.3)
    phi = si.wilson_vector(rng, dims, nc, 2)
    d = wilson_dense(U, m, True)
    f = phi.reshape(-1, 2)
    chi = np.linalg.solve(d.conj().T @ d, f).reshape(phi.shape)
    psi = wilson_apply(U, chi, m)
    g = -2.0 * wilson_force(U, psi, chi, True)
    force = project_su(U, g)
    np.testing.assert_allclose(force, np.conj(np.swapaxes(force, -1, -2)), atol=1e-13)
    np.testing.assert_allclose(np.trace(force, axis1=-2, axis2=-1), 0, atol=1e-13)
    dirs = si.su_n_directions(np.random.default_rng(1), dims, nc, 5)
    eps = 1e-6
    for h in dirs:
        w, v = np.linalg.eigh(h)
        expo = lambda s: (v * np.exp(1j * s * w)[..., None, :]) @ np.conj(np.swapaxes(v, -1, -2))
        lp = _solve_loss(expo(eps) @ U, phi, m)
        ln = _solve_loss(expo(-eps) @ U, phi, m)
        fd = (lp - ln) / (2 * eps)
        an = np.real(np.sum(np.trace(h @ force, axis1=-2, axis2=-1)))
        assert abs(fd - an) < 1e-6 * max(1.0, abs(an))
    # grad_phi = 2 chi (torch convention) by differences in Re and Im of one component
    for idx in [(0, 0, 0, 0, 1, 2, 1), (3, 1, 0, 1, 0, 0, 0)]:
        for unit in (1.0, 1j):
            pp, pn = phi.copy(), phi.copy()
            pp[idx] += eps * unit
            pn[idx] -= eps * unit
            fd = (_solve_loss(U, pp, m) - _solve_loss(U, pn, m)) / (2 * eps)
            expect = (2 * chi[idx]).real if unit == 1.0 else (2 * chi[idx]).imag
            assert abs(fd - expect) < 1e-6 * max(1.0, abs(expect))
