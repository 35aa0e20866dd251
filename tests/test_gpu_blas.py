"""GPU parity of the multi-RHS BLAS-1 kernels (Sec. 3) against NumPy on the same stored values."""
import numpy as np
import pytest
import torch

import synthetic_inputs as si
from paper_2112_14640_amd import dirac
from tests.gpu_helpers import bf16_pairs_to_host, host, round_bf16, round_c64, to_bf16_pairs, to_dev

pytestmark = pytest.mark.gpu


def _dev(a, prec):
    if prec == "fp64":
        return to_dev(a), a
    if prec == "fp32":
        return to_dev(a, torch.complex64), round_c64(a)
    return to_bf16_pairs(a), round_bf16(a)


def _host(t, prec):
    return bf16_pairs_to_host(t) if prec == "bf16" else host(t).astype(np.complex128)


SHAPES = [(7, 1), (33, 5), (1000, 12), (40000, 12), (3, 256), (257, 24)]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("shape", SHAPES)
def test_norm2_and_dot(prec, shape):
    rng = np.random.default_rng(1)
    x = si.complex_gaussian(rng, shape)
    y = si.complex_gaussian(rng, shape)
    xd, xv = _dev(x, prec)
    yd, yv = _dev(y, prec)
    n = host(dirac.norm2(xd))
    np.testing.assert_allclose(n, np.sum(np.abs(xv) ** 2, axis=0), rtol=1e-12)
    d = host(dirac.dot(xd, yd))
    np.testing.assert_allclose(d, np.sum(np.conj(xv) * yv, axis=0), rtol=1e-11, atol=1e-11 * np.sqrt(shape[0]))
    # fixed summation order: bitwise reproducible
    assert np.array_equal(host(dirac.norm2(xd)), n)


@pytest.mark.parametrize("px,py", [("fp64", "fp64"), ("fp32", "fp32"), ("fp32", "fp64"), ("bf16", "fp32"),
                                   ("fp64", "bf16")])
def test_caxpy_cxpay(px, py):
    rng = np.random.default_rng(2)
    shape = (2049, 12)
    x = si.complex_gaussian(rng, shape)
    y = si.complex_gaussian(rng, shape)
    a = si.complex_gaussian(rng, (12,))
    xd, xv = _dev(x, px)
    yd, yv = _dev(y, py)
    dirac.caxpy(torch.from_numpy(a), xd, yd)
    expect = yv + a * xv
    tol = {"fp64": 1e-14, "fp32": 1e-6, "bf16": 8e-3}[py]
    np.testing.assert_allclose(_host(yd, py), expect, rtol=0, atol=tol * 4)
    yd2, yv2 = _dev(y, py)
    dirac.cxpay(xd, torch.from_numpy(a), yd2)
    np.testing.assert_allclose(_host(yd2, py), xv + a * yv2, rtol=0, atol=tol * 4)


def test_cast_round_to_nearest_even():
    rng = np.random.default_rng(3)
    x = si.complex_gaussian(rng, (5000, 3)) * 10.0 ** rng.uniform(-20, 20, (5000, 3))
    xd = to_dev(x)
    x32 = dirac.cast(xd, "fp32")
    assert np.array_equal(host(x32), x.astype(np.complex64))
    xb = dirac.cast(x32, "bf16")
    ref = torch.view_as_real(torch.from_numpy(x.astype(np.complex64))).to(torch.bfloat16)
    assert torch.equal(xb.cpu().view(torch.int16), ref.view(torch.int16))
    back = dirac.cast(xb, "fp64")
    np.testing.assert_array_equal(host(back), round_bf16(x))


def test_gamma5_and_epsilon():
    rng = np.random.default_rng(4)
    dims = (4, 2, 6, 4)
    nx, ny, nz, nt = dims
    psi = si.wilson_vector(rng, dims, 3, 5)
    out = host(dirac.gamma5("wilson", to_dev(psi)))
    np.testing.assert_array_equal(out, psi * np.array([1, 1, -1, -1])[:, None])
    phi = si.staggered_vector(rng, dims, 3, 5)
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    eps = np.where((x + y + z + t) % 2 == 0, 1.0, -1.0)[..., None, None]
    np.testing.assert_array_equal(host(dirac.gamma5("staggered", to_dev(phi))), phi * eps)


def test_measurement_probes():
    """The copy, FMA and row-gather probes (their own library) return sane, finite rates; the copy copies, and the
    row gather writes the exclusive or of each row and its six +-y, +-z, +-t neighbour rows."""
    from paper_2112_14640_amd import measure

    src = torch.randn(2 ** 22, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    bw = measure.copy_rate(src, dst, reps=3)
    assert torch.equal(src, dst)
    assert 1e11 < bw < 2e13, bw
    for prec in ("fp32", "fp64"):
        f = measure.fma_rate(prec)
        assert 1e12 < f < 4e14, (prec, f)
    with pytest.raises(ValueError):
        measure.copy_rate(src, dst[:-1])
    dims, site_bytes = (6, 4, 8, 6), 48
    nx, ny, nz, nt = dims
    a = torch.randint(0, 2 ** 31 - 1, (nt, nz, ny, nx, site_bytes // 4), dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    r = measure.row_gather_rate(dims, site_bytes, a, b, reps=2)
    assert 1e9 < r < 2e13, r
    h = a.cpu()
    want = h.clone()
    for axis in (0, 1, 2):  # t, z, y
        for s in (1, -1):
            want ^= torch.roll(h, s, dims=axis)
    assert torch.equal(b.cpu(), want)
    measure.row_gather_rate(dims, site_bytes, a, b, reps=1, nrows=1)
    assert torch.equal(b, a)
    with pytest.raises(ValueError):
        measure.row_gather_rate((6, 4, 6, 6), site_bytes, a, b)  # nz not a multiple of 4
