"""Pins for the oracle solvers: dense solves, exit rules, Lanczos spectrum estimate."""
import numpy as np

import synthetic_inputs as si
from oracle.brillouin import brillouin_apply, brillouin_links
from oracle.dense import staggered_dense, wilson_dense
from oracle.solvers import bicgstab, cg, lanczos_extremes, norm2
from oracle.staggered import staggered_apply, staggered_apply_dagger
from oracle.wilson import wilson_apply, wilson_apply_dagger


def _cols(f):
    return f.reshape(-1, f.shape[-1])


def test_cg_wilson_normal_equals_dense_solve():
    dims, nc, m = (4, 4, 4, 4), 3, 0.1
    rng = np.random.default_rng(31)
    U = si.gauge_field(rng, dims, nc, "near", 0.5)
    b = si.wilson_vector(rng, dims, nc, 3)
    a = lambda x: wilson_apply_dagger(U, wilson_apply(U, x, m), m)
    res = cg(a, b, tol=1e-12, maxit=2000)
    assert res.status == "converged"
    assert np.all(res.true_relres < 1e-12)
    d = wilson_dense(U, m, True)
    x = np.linalg.solve(d.conj().T @ d, _cols(b))
    np.testing.assert_allclose(_cols(res.x), x, rtol=0, atol=1e-9 * np.abs(x).max())


def test_cg_staggered_equals_dense_solve():
    dims, nc, m = (4, 4, 2, 4), 3, 0.05
    rng = np.random.default_rng(32)
    U = si.gauge_field(rng, dims, nc, "haar")
    b = si.staggered_vector(rng, dims, nc, 2)
    a = lambda x: staggered_apply_dagger(U, staggered_apply(U, x, m), m)
    res = cg(a, b, tol=1e-12, maxit=5000)
    assert res.status == "converged"
    d = staggered_dense(U, m, True)
    x = np.linalg.solve(d.conj().T @ d, _cols(b))
    np.testing.assert_allclose(_cols(res.x), x, atol=1e-8 * np.abs(x).max())


def test_bicgstab_wilson_and_brillouin_equal_dense_solve():
    dims, nc, m = (2, 2, 2, 4), 2, 0.1
    rng = np.random.default_rng(33)
    U = si.gauge_field(rng, dims, nc, "haar")
    b = si.wilson_vector(rng, dims, nc, 3)
    res = bicgstab(lambda x: wilson_apply(U, x, m), b, tol=1e-12, maxit=2000)
    assert res.status == "converged" and np.all(res.true_relres < 1e-12)
    x = np.linalg.solve(wilson_dense(U, m, True), _cols(b))
    np.testing.assert_allclose(_cols(res.x), x, atol=1e-9 * np.abs(x).max())
    w40 = brillouin_links(U)
    res = bicgstab(lambda x: brillouin_apply(w40, x, m), b, tol=1e-12, maxit=2000)
    assert res.status == "converged" and np.all(res.true_relres < 1e-12)


def test_exit_rules():
    dims, nc, m = (2, 2, 2, 4), 2, 0.01
    rng = np.random.default_rng(34)
    U = si.gauge_field(rng, dims, nc, "haar")
    b = si.wilson_vector(rng, dims, nc, 2)
    a = lambda x: wilson_apply_dagger(U, wilson_apply(U, x, m), m)
    assert cg(a, b, tol=1e-12, maxit=1).status == "maxit"
    # single-precision arithmetic stagnates: the 1 % gap between updated and recomputed residual ends the solve
    a32 = lambda x: a(x.astype(np.complex64)).astype(np.complex64).astype(np.complex128)
    res = cg(a32, b, tol=1e-14, maxit=5000, recompute_every=20)
    assert res.status == "stagnated"
    assert 1e-9 < res.true_relres.max() < 1e-3
    # zero right-hand side: nothing to do
    res = cg(a, np.zeros_like(b), tol=1e-10)
    assert res.status == "converged" and res.iterations == 0


def test_lanczos_extremes_match_dense_spectrum():
    dims, nc, m = (4, 4, 4, 4), 1, 0.2
    rng = np.random.default_rng(35)
    U = si.gauge_field(rng, dims, nc, "near", 0.5)
    b = si.wilson_vector(rng, dims, nc, 1)
    a = lambda x: wilson_apply_dagger(U, wilson_apply(U, x, m), m)
    res = cg(a, b, tol=1e-12, maxit=3000, recompute_every=10 ** 9)
    lo, hi = lanczos_extremes([al[0] for al in res.alphas], [bt[0] for bt in res.betas])
    d = wilson_dense(U, m, True)
    ev = np.linalg.eigvalsh(d.conj().T @ d)
    assert abs(hi - ev[-1]) / ev[-1] < 1e-3
    assert abs(lo - ev[0]) / ev[0] < 2e-2
