"""GPU link gradients and the autograd front end against the oracle and finite differences."""
import numpy as np
import pytest
import torch

import synthetic_inputs as si
from oracle.dense import wilson_dense
from oracle.force import project_su, staggered_force, wilson_force
from oracle.wilson import wilson_apply
from paper_2112_14640_amd import autograd as dag
from paper_2112_14640_amd import dirac
from tests.gpu_helpers import host, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("op", ["wilson", "staggered"])
@pytest.mark.parametrize("apbc", [True, False])
def test_force_matches_oracle(op, apbc):
    dims, nc, nv = (4, 2, 6, 4), 3, 3
    rng = np.random.default_rng(21)
    U = si.gauge_field(rng, dims, nc, "haar")
    mk = si.staggered_vector if op == "staggered" else si.wilson_vector
    psi, chi = mk(rng, dims, nc, nv), mk(rng, dims, nc, nv)
    g = host(dirac.force(op, to_dev(U), to_dev(psi), to_dev(chi), 1.0, apbc))
    ref = (staggered_force if op == "staggered" else wilson_force)(U, psi, chi, apbc)
    assert np.max(np.abs(g - ref)) < 1e-12 * np.max(np.abs(ref))
    g2 = host(dirac.force(op, to_dev(U), to_dev(psi), to_dev(chi), -2.5, apbc, out=to_dev(g)))
    np.testing.assert_allclose(g2, -1.5 * ref, atol=1e-12)


def test_project_su_matches_oracle():
    rng = np.random.default_rng(22)
    U = si.haar_su_n(rng, (50,), 3)
    g = si.complex_gaussian(rng, (50, 3, 3))
    F = host(dirac.project_su(to_dev(U), to_dev(g)))
    np.testing.assert_allclose(F, project_su(U, g), atol=1e-14)


def test_apply_backward_matches_adjoint_and_force():
    dims, nc, nv = (4, 4, 2, 4), 3, 2
    rng = np.random.default_rng(23)
    U = si.gauge_field(rng, dims, nc, "haar")
    u = si.wilson_vector(rng, dims, nc, nv)
    w = si.wilson_vector(rng, dims, nc, nv)
    Ud = to_dev(U).requires_grad_(True)
    ud = to_dev(u).requires_grad_(True)
    v = dag.apply("wilson", Ud, ud, 0.1)
    loss = torch.sum((torch.conj(to_dev(w)) * v).real)
    loss.backward()
    # d Re<w, D u> : grad_u = D^dag w, grad_U = force(w, u)
    from oracle.wilson import wilson_apply_dagger
    np.testing.assert_allclose(host(ud.grad), wilson_apply_dagger(U, w, 0.1), atol=1e-12)
    np.testing.assert_allclose(host(Ud.grad), wilson_force(U, w, u, True), atol=1e-12)


def test_torch_gradcheck_small():
    """torch.autograd.gradcheck of DiracApply in FP64 on a 2^4 lattice (finite differences by torch)."""
    dims, nc, nv = (2, 2, 2, 2), 2, 1
    rng = np.random.default_rng(24)
    U = to_dev(si.gauge_field(rng, dims, nc, "haar")).requires_grad_(True)
    u = to_dev(si.wilson_vector(rng, dims, nc, nv)).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: dag.apply("wilson", a, b, 0.2), (U, u), eps=1e-6, atol=1e-7,
                                    rtol=1e-5, fast_mode=True)


def test_solve_gradients_against_oracle_4x4():
    """L = sum_i Re phi_i^dag (D^dag D)^{-1} phi_i: grads vs the oracle's formula on 4^4 (dense solve)."""
    dims, nc, nv, m = (4, 4, 4, 4), 3, 2, 0.2
    rng = np.random.default_rng(25)
    U = si.gauge_field(rng, dims, nc, "near", 0.3)
    phi = si.wilson_vector(rng, dims, nc, nv)
    Ud = to_dev(U).requires_grad_(True)
    pd = to_dev(phi).requires_grad_(True)
    x = dag.solve_normal("wilson", Ud, pd, m, tol=1e-13, maxit=5000)
    loss = torch.sum((torch.conj(pd) * x).real)
    loss.backward()
    d = wilson_dense(U, m, True)
    chi = np.linalg.solve(d.conj().T @ d, phi.reshape(-1, nv)).reshape(phi.shape)
    np.testing.assert_allclose(host(pd.grad), 2 * chi, atol=1e-9)
    g_ref = -2.0 * wilson_force(U, wilson_apply(U, chi, m), chi, True)
    np.testing.assert_allclose(host(Ud.grad), g_ref, atol=1e-9 * np.max(np.abs(g_ref)))
    F = host(dag.su_force(Ud.detach(), Ud.grad))
    np.testing.assert_allclose(F, project_su(U, g_ref), atol=1e-9 * np.max(np.abs(g_ref)))
