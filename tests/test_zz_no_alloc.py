"""dirac_dot_noalloc (the dot product whose reduction partials live in library-owned static device memory)
against dirac_dot with a caller workspace, through the C ABI: the same kernels in the same order, so the
results agree bit for bit.  Two calls in a row, the second on a smaller input (fewer rows and fewer
right-hand sides), so stale partials of the first call would show; then the size limit."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2112_14640_amd import _lib as L
from tests.gpu_helpers import DEV

pytestmark = pytest.mark.gpu


def _vec(rng, nrows, nv, dtype):
    a = (rng.standard_normal((nrows, nv)) + 1j * rng.standard_normal((nrows, nv))) / np.sqrt(2)
    return torch.from_numpy(a).to(DEV).to(dtype).contiguous()


def _dot_ws(lib, prec, x, y, nrows, nv, stream):
    out = torch.empty(2 * nv, dtype=torch.float64, device=DEV)
    nbytes = lib.dirac_blas_workspace_bytes(nv)
    ws = torch.empty(nbytes // 8, dtype=torch.float64, device=DEV)
    L.check(lib.dirac_dot(prec, x.data_ptr(), prec, y.data_ptr(), nrows, nv, out.data_ptr(), ws.data_ptr(), nbytes,
                          stream), "dirac_dot")
    return out


def _dot_noalloc(lib, prec, x, y, nrows, nv, stream):
    out = torch.empty(2 * nv, dtype=torch.float64, device=DEV)
    L.check(lib.dirac_dot_noalloc(prec, x.data_ptr(), prec, y.data_ptr(), nrows, nv, out.data_ptr(), stream),
            "dirac_dot_noalloc")
    return out


@pytest.mark.parametrize("prec,dtype", [(L.FP64, torch.complex128), (L.FP32, torch.complex64)])
def test_noalloc_dot_matches_workspace_dot(prec, dtype):
    lib = L.load()
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(77)
    for nrows, nv in ((40000, 24), (999, 5)):  # the second call is smaller in both rows and RHS
        x, y = _vec(rng, nrows, nv, dtype), _vec(rng, nrows, nv, dtype)
        a = _dot_noalloc(lib, prec, x, y, nrows, nv, stream)
        b = _dot_ws(lib, prec, x, y, nrows, nv, stream)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (nrows, nv)
        ref = (torch.conj(x.to(torch.complex128)) * y.to(torch.complex128)).sum(0)
        got = torch.view_as_complex(a.view(nv, 2))
        assert torch.allclose(got, ref, rtol=1e-12, atol=1e-9 * nrows), (nrows, nv)


def test_noalloc_dot_rejects_too_many_rhs():
    lib = L.load()
    x = torch.zeros((4, 257), dtype=torch.complex128, device=DEV)
    out = torch.zeros(2 * 257, dtype=torch.float64, device=DEV)
    st = lib.dirac_dot_noalloc(L.FP64, x.data_ptr(), L.FP64, x.data_ptr(), 4, 257, out.data_ptr(),
                               torch.cuda.current_stream().cuda_stream)
    assert st == L.EINVAL
    assert b"256" in lib.dirac_last_error() or b"nv" in lib.dirac_last_error()
