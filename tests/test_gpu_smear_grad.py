"""GPU stout smearing and the differentiation of the Brillouin operator through W -> V -> U, against the
oracle (FP64).

* stout steps element by element against ``oracle.stout``;
* every backward (stout step, W(V) path averages, the Brillouin link force) against central differences
  of the oracle's forward functions along random complex directions E: dL/d eps = Re sum tr(G^+ E);
* end to end, U -> stout -> V -> W -> D_B u (and through a CG solve on D_B^+ D_B) by torch.autograd over
  the library's backward kernels, against central differences of the oracle chain.
"""
import numpy as np
import pytest
import torch

import synthetic_inputs as si
from oracle.brillouin import brillouin_apply, brillouin_links
from oracle.dense import brillouin_dense
from oracle.brillouin import brillouin_links_all
from oracle.stout import stout_smear, stout_step
from paper_2112_14640_amd import autograd as ag
from paper_2112_14640_amd import dirac
from tests.gpu_helpers import host, to_dev

pytestmark = pytest.mark.gpu


def _cg(rng, shape):
    return si.complex_gaussian(rng, shape)


def _rdot(g, e):
    """Re sum conj(g) e: the directional derivative of L along E given G = dL/dRe + i dL/dIm."""
    return float(np.sum(np.conj(g) * e).real)


@pytest.mark.parametrize("nc", [2, 3, 4])
def test_stout_forward_matches_oracle(nc):
    dims = (4, 2, 4, 6)
    rng = np.random.default_rng(600 + nc)
    U = si.gauge_field(rng, dims, nc, "haar")
    V1 = host(dirac.stout_step(to_dev(U), 0.12))
    assert np.max(np.abs(V1 - stout_step(U, 0.12))) < 1e-13
    V3 = host(dirac.stout_smear(to_dev(U), 0.12, 3))
    assert np.max(np.abs(V3 - stout_smear(U, 0.12, 3))) < 1e-13


def _fd(fn, x, e, eps=1e-6):
    return (fn(x + eps * e) - fn(x - eps * e)) / (2 * eps)


@pytest.mark.parametrize("nc", [2, 3])
def test_stout_backward_against_differences(nc):
    dims, rho = (2, 4, 2, 4), 0.12
    rng = np.random.default_rng(610 + nc)
    U = si.gauge_field(rng, dims, nc, "near", 0.6)
    R = _cg(rng, U.shape)
    gU = host(dirac.stout_backward(to_dev(U), to_dev(R), rho))
    for k in range(4):
        E = _cg(np.random.default_rng(620 + k), U.shape)
        want = _fd(lambda u: float(np.sum(np.conj(R) * stout_step(u, rho)).real), U, E)
        assert abs(_rdot(gU, E) - want) < 1e-7 * max(1.0, abs(want)), (k, _rdot(gU, E), want)


@pytest.mark.parametrize("nc", [2, 3])
def test_links_backward_against_differences(nc):
    dims = (2, 2, 4, 4)
    rng = np.random.default_rng(630 + nc)
    V = si.gauge_field(rng, dims, nc, "haar")
    R = _cg(rng, dims[::-1] + (40, nc, nc))
    gV = host(dirac.brillouin_links_backward(to_dev(V), to_dev(R)))
    for k in range(4):
        E = _cg(np.random.default_rng(640 + k), V.shape)
        want = _fd(lambda v: float(np.sum(np.conj(R) * brillouin_links(v)).real), V, E)
        assert abs(_rdot(gV, E) - want) < 1e-7 * max(1.0, abs(want)), (k, _rdot(gV, E), want)


@pytest.mark.parametrize("apbc", [True, False])
def test_brillouin_force_against_differences(apbc):
    """g = d Re(psi^+ D_B(W) chi)/dW: L is linear in W, so the central difference is exact."""
    dims, nc, nv, m = (2, 4, 2, 4), 3, 3, 0.1
    rng = np.random.default_rng(650)
    W = brillouin_links(si.gauge_field(rng, dims, nc, "haar"))
    psi = si.wilson_vector(rng, dims, nc, nv)
    chi = si.wilson_vector(rng, dims, nc, nv)
    g = host(dirac.force("brillouin", to_dev(W), to_dev(psi), to_dev(chi), 1.0, apbc))
    for k in range(4):
        E = _cg(np.random.default_rng(660 + k), W.shape)

        def L(w):
            return float(np.sum(np.conj(psi) * brillouin_apply(w, chi, m, apbc)).real)

        want = _fd(L, W, E, eps=0.5)
        assert abs(_rdot(g, E) - want) < 1e-10 * max(1.0, abs(want)), (k, _rdot(g, E), want)


def _chain_oracle(U, u, m, rho, steps, R):
    V = stout_smear(U, rho, steps)
    return float(np.sum(np.conj(R) * brillouin_apply(brillouin_links(V), u, m)).real)


def test_end_to_end_apply_gradient():
    """U -> stout (2 steps) -> W -> D_B u -> L = Re sum conj(R) D_B u: torch.autograd over the library
    against central differences of the oracle chain, for the links and for u."""
    dims, nc, nv, m, rho = (2, 2, 2, 4), 2, 2, 0.1, 0.12
    rng = np.random.default_rng(670)
    U = si.gauge_field(rng, dims, nc, "near", 0.5)
    u = si.wilson_vector(rng, dims, nc, nv)
    R = si.wilson_vector(rng, dims, nc, nv)
    Ud = to_dev(U).requires_grad_(True)
    ud = to_dev(u).requires_grad_(True)
    W = ag.brillouin_links(ag.stout_smear(Ud, rho, 2))
    v = ag.apply("brillouin", W, ud, m)
    loss = (torch.conj(to_dev(R)) * v).real.sum()
    loss.backward()
    gU, gu = host(Ud.grad), host(ud.grad)
    for k in range(3):
        E = _cg(np.random.default_rng(680 + k), U.shape)
        want = _fd(lambda x: _chain_oracle(x, u, m, rho, 2, R), U, E)
        assert abs(_rdot(gU, E) - want) < 1e-6 * max(1.0, abs(want)), (k, _rdot(gU, E), want)
    e = _cg(np.random.default_rng(690), u.shape)
    want = _fd(lambda x: _chain_oracle(U, x, m, rho, 2, R), u, e, eps=0.5)
    assert abs(_rdot(gu, e) - want) < 1e-9 * max(1.0, abs(want))


def test_solve_gradient_brillouin():
    """L = Re sum phi^+ (D_B^+ D_B)^{-1} phi with D_B built from W(V): the gradient with respect to V through
    the adjoint solve and the link backward, against central differences of a dense oracle solve."""
    dims, nc, nv, m = (2, 2, 2, 2), 2, 2, 0.3
    rng = np.random.default_rng(700)
    V = si.gauge_field(rng, dims, nc, "near", 0.5)
    phi = si.wilson_vector(rng, dims, nc, nv)
    Vd = to_dev(V).requires_grad_(True)
    W = ag.brillouin_links(Vd)
    x = ag.solve_normal("brillouin", W, to_dev(phi), m, tol=1e-13, maxit=5000)
    loss = (torch.conj(to_dev(phi)) * x).real.sum()
    loss.backward()
    gV = host(Vd.grad)
    cols = phi.reshape(-1, nv)

    def L(v):
        d = brillouin_dense(brillouin_links_all(v), dims, m)
        xs = np.linalg.solve(d.conj().T @ d, cols)
        return float(np.sum(np.conj(cols) * xs).real)

    for k in range(3):
        E = _cg(np.random.default_rng(710 + k), V.shape)
        want = _fd(L, V, E)
        assert abs(_rdot(gV, E) - want) < 1e-6 * max(1.0, abs(want)), (k, _rdot(gV, E), want)
