"""CG on D_W^dagger D_W at 32^3x64 (Nc=3, Nv=12, m=0.01, links exp(i 0.5 H)) to a true relative residual of
1e-10: plain FP64, and FP32 / BF16-storage inner solvers inside the FP64 outer loop, with reliable updates
(residual replacement factor delta = 0.1, and 0.01) and with defect correction.

The oracle recomputes r = b - D^dagger D x in FP64 at 2000 sampled sites (plus the t-boundary slices) from
host copies of the links and of each solution: D x on the sites and their eight neighbours, then D^dagger at
the sites.  The bar on that sampled relative residual is 1e-9: the library's stopping rule bounds the
whole-lattice ratio by 1e-10, and the ratio over a random sample of 2000 sites (about 290k complex entries
per RHS) differs from the whole-lattice one by a few per cent, so 1e-9 leaves a tenfold margin and still
fails for any solution an order of magnitude short of the goal.  The mixed solutions are also compared
with the FP64 one.
"""
import gc

import numpy as np
import pytest
import torch

import synthetic_inputs as si
from oracle.wilson import wilson_apply, wilson_apply_dagger
from paper_2112_14640_amd import dirac
from tests.gpu_helpers import DEV, host, sample_sites

pytestmark = pytest.mark.gpu

CFG = si.config("cg_32x64")


@pytest.fixture(scope="module")
def problem():
    nx, ny, nz, nt = CFG["dims"]
    gen = torch.Generator(device=DEV).manual_seed(CFG["seed"] + 300)
    U = si.near_identity_su_n_t(gen, (nt, nz, ny, nx, 4), CFG["nc"], CFG["spread"], DEV)
    b = si.complex_gaussian_t(gen, (nt, nz, ny, nx, CFG["nc"], 4, CFG["nv"]), DEV)
    state = {"U": U, "b": b, "Uh": host(U), "bh": host(b)}
    yield state
    state.clear()
    gc.collect()
    torch.cuda.empty_cache()


def _oracle_residual_at(Uh, xh, bh, mass, sites):
    """Per-RHS ||b - D^dag D x|| / ||b|| over the sampled sites, all in FP64 by the oracle."""
    nx, ny, nz, nt = CFG["dims"]
    ext = np.array([nx, ny, nz, nt])
    near = [sites]
    for mu in range(4):
        e = np.zeros(4, dtype=np.int64)
        e[mu] = 1
        near += [np.mod(sites + e, ext), np.mod(sites - e, ext)]
    near = np.unique(np.concatenate(near), axis=0)
    y = np.zeros(xh.shape, dtype=np.complex128)  # D x is only needed next to the sampled sites
    y[near[:, 3], near[:, 2], near[:, 1], near[:, 0]] = wilson_apply(Uh, xh, mass, True, sites=near)
    ax = wilson_apply_dagger(Uh, y, mass, True, sites=sites)
    bs = bh[sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0]]
    num = np.linalg.norm((bs - ax).reshape(-1, bh.shape[-1]), axis=0)
    return num / np.linalg.norm(bs.reshape(-1, bh.shape[-1]), axis=0)


def _fp64_solution(problem):
    if "x64" not in problem:
        x64, info = dirac.cg("wilson", problem["U"], problem["b"], CFG["mass"], tol=1e-10, maxit=20000)
        assert info.reason == "converged", info
        problem["x64"] = x64
    return problem["x64"]


CASES = [
    ("fp64", None),
    ("fp32", dict(mixed_scheme=0, delta=0.1)),
    ("bf16", dict(mixed_scheme=0, delta=0.1)),
    # the setting that once diverged (the inner BF16 recurrence grew without bound): regression test
    ("bf16", dict(mixed_scheme=0, delta=0.01)),
    ("fp32", dict(mixed_scheme=1)),
]


@pytest.mark.parametrize("inner,opts", CASES, ids=["fp64", "fp32-ru0.1", "bf16-ru0.1", "bf16-ru0.01", "fp32-dc"])
def test_cg_32x64_true_residual(problem, inner, opts):
    U, b = problem["U"], problem["b"]
    m = CFG["mass"]
    kw = {} if inner == "fp64" else dict(inner=inner, gauge_lo=U.to(torch.complex64), opts=opts)
    x, info = dirac.cg("wilson", U, b, m, tol=1e-10, maxit=20000, **kw)
    assert info.reason == "converged", info
    assert max(info.true_relres) < 1e-10, info.true_relres
    sites = sample_sites(CFG["dims"], 2000, seed=31)
    res = _oracle_residual_at(problem["Uh"], host(x), problem["bh"], m, sites)
    assert np.all(res < 1e-9), res
    if inner != "fp64":
        x64 = _fp64_solution(problem)
        d = torch.linalg.vector_norm((x - x64).reshape(-1, CFG["nv"]), dim=0)
        rel = (d / torch.linalg.vector_norm(x64.reshape(-1, CFG["nv"]), dim=0)).max().item()
        assert rel < 1e-6, rel
