"""Parity at scale: Brillouin and staggered at 48^3x96 (Nc=3, Nv=12, FP32, Haar links, m=0.05), Wilson at
32^3x64 for Nc in {2, 4} x Nv in {1, 4, 12, 24}, and mixed-precision BiCGstab on D_B at 32^3x64 to 1e-8.

Inputs are drawn on the device from seeded torch generators (the host could not draw 10^7 Haar links
in reasonable time).  The oracle then evaluates sampled output sites in FP64 from host copies of the
same FP32-rounded inputs; Brillouin links are rebuilt by the oracle from the 4 links per site at the
sampled sites only (the 40-direction array is 30 GB at 48^3x96).
"""
import gc

import numpy as np
import pytest
import torch

import synthetic_inputs as si
from oracle.brillouin import brillouin_apply_sites, brillouin_links_all
from oracle.staggered import staggered_apply, staggered_apply_dagger
from oracle.wilson import wilson_apply, wilson_apply_dagger
from paper_2112_14640_amd import dirac
from tests.gpu_helpers import DEV, host, parity, sample_sites

pytestmark = pytest.mark.gpu

MASS = 0.05


def _gen(seed):
    return torch.Generator(device=DEV).manual_seed(seed)


def _haar_links(dims, nc, seed, dtype=torch.complex64):
    nx, ny, nz, nt = dims
    return si.haar_su_n_t(_gen(seed), (nt, nz, ny, nx, 4), nc, DEV, dtype)


def _spinor(dims, nc, nv, seed, spin=True, dtype=torch.complex64):
    nx, ny, nz, nt = dims
    shape = (nt, nz, ny, nx, nc, 4, nv) if spin else (nt, nz, ny, nx, nc, nv)
    return si.complex_gaussian_t(_gen(seed), shape, DEV, dtype)


def _at(t, sites):
    s = torch.as_tensor(sites, device=t.device)
    return host(t[s[:, 3], s[:, 2], s[:, 1], s[:, 0]]).astype(np.complex128)


def _free():
    gc.collect()
    torch.cuda.empty_cache()


def test_brillouin_48x96_nv12_fp32_sampled():
    dims = (48, 48, 48, 96)
    U = _haar_links(dims, 3, 501)
    W = dirac.brillouin_links(U)
    u = _spinor(dims, 3, 12, 502)
    sites = sample_sites(dims, 64, seed=5)
    got = {dag: _at((dirac.apply_dagger if dag else dirac.apply)("brillouin", W, u, MASS), sites)
           for dag in (False, True)}
    w_dev = _at(W, sites)
    del W
    _free()
    Uh, uh = host(U), host(u)
    w81 = brillouin_links_all(Uh, sites=sites)
    assert np.max(np.abs(w_dev - w81[:, :40])) < 2e-6
    for dag in (False, True):
        ref = brillouin_apply_sites(w81, uh, MASS, sites, True, dagger=dag)
        parity(got[dag], ref, 1e-5, dag)
    del U, u, Uh, uh
    _free()


def test_staggered_48x96_nv12_fp32_sampled():
    dims = (48, 48, 48, 96)
    U = _haar_links(dims, 3, 511)
    u = _spinor(dims, 3, 12, 512, spin=False)
    sites = sample_sites(dims, 400, seed=6)
    got = {dag: _at((dirac.apply_dagger if dag else dirac.apply)("staggered", U, u, MASS), sites)
           for dag in (False, True)}
    Uh, uh = host(U), host(u)
    for dag, fn in ((False, staggered_apply), (True, staggered_apply_dagger)):
        parity(got[dag], fn(Uh, uh, MASS, True, sites=sites), 1e-5, dag)
    del U, u, Uh, uh
    _free()


@pytest.mark.parametrize("nv", [1, 4, 12, 24])
@pytest.mark.parametrize("nc", [2, 4])
def test_wilson_32x64_nc_nv_fp32_sampled(nc, nv):
    dims = (32, 32, 32, 64)
    U = _haar_links(dims, nc, 520 + nc)
    u = _spinor(dims, nc, nv, 530 + nv)
    sites = sample_sites(dims, 400, seed=7)
    got = {dag: _at((dirac.apply_dagger if dag else dirac.apply)("wilson", U, u, MASS), sites)
           for dag in (False, True)}
    Uh, uh = host(U), host(u)
    for dag, fn in ((False, wilson_apply), (True, wilson_apply_dagger)):
        parity(got[dag], fn(Uh, uh, MASS, True, sites=sites), 1e-5, (nc, nv, dag))
    del U, u, Uh, uh
    _free()


def test_bicgstab_brillouin_32x64_mixed_to_1e8():
    """BiCGstab on D_B (Haar links, m=0.05, Nv=12) with an FP32 inner solver inside the FP64 outer
    loop; the FP64 residual is recomputed by the library and by the oracle at sampled sites."""
    dims = (32, 32, 32, 64)
    U64 = _haar_links(dims, 3, 541, torch.complex128)
    W64 = dirac.brillouin_links(U64)
    W32 = W64.to(torch.complex64)
    b = _spinor(dims, 3, 12, 542, dtype=torch.complex128)
    x, info = dirac.bicgstab("brillouin", W64, b, MASS, tol=1e-8, maxit=3000, inner="fp32", gauge_lo=W32)
    assert info.reason == "converged", info
    assert max(info.true_relres) < 1e-8
    # the oracle's D_B x at sampled sites, with links rebuilt from U64 there
    r_dev = dirac.apply("brillouin", W64, x, MASS)
    sites = sample_sites(dims, 48, seed=8)
    dx_dev, b_s = _at(r_dev, sites), _at(b, sites)
    del W64, W32, r_dev
    _free()
    w81 = brillouin_links_all(host(U64), sites=sites)
    dx_ref = brillouin_apply_sites(w81, host(x), MASS, sites, True)
    parity(dx_dev, dx_ref, 1e-12)
    # residual at the sampled sites against b there: of the size of the global relative residual
    res = np.linalg.norm((b_s - dx_ref).reshape(-1, 12), axis=0) / np.linalg.norm(b_s.reshape(-1, 12), axis=0)
    assert np.all(res < 1e-6), res
    del U64, b, x
    _free()
