"""Measurement probes of the device (libdirac_probe.so, include/dirac_probe.h).

Not part of the method: the sustained copy bandwidth and FMA rate that the roofline figures print
next to the published peaks, and the stencils' row-gather access pattern without their arithmetic.
The library is built by ``paper_2112_14640_amd.build`` beside the operator library and shares no
code with it.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdirac_probe.so")

_lib = None
_SIGS = {
    "dirac_probe_copy": [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.POINTER(C.c_double), C.c_void_p],
    "dirac_probe_fma": [C.c_int, C.c_void_p, C.POINTER(C.c_double), C.c_void_p],
    "dirac_probe_row_gather": [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                               C.c_int, C.POINTER(C.c_double), C.c_void_p],
}


def load():
    """Load libdirac_probe.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2112_14640_amd.build` first")
    lib = C.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = C.c_int
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc == -1:
        raise ValueError(f"{what}: bad arguments")
    if rc != 0:
        raise RuntimeError(f"{what}: HIP error ({rc})")


def _dev(t: torch.Tensor, name: str):
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous device tensor")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def copy_rate(src: torch.Tensor, dst: torch.Tensor, reps: int = 10) -> float:
    """Sustained device copy rate (read + written bytes per second) over src -> dst (same byte size)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or dst.device != src.device:
        raise ValueError("copy_rate: src and dst must have the same byte size and device")
    out = C.c_double(0.0)
    _check(load().dirac_probe_copy(_dev(src, "src"), _dev(dst, "dst"), nbytes, reps, C.byref(out), _stream()),
           "dirac_probe_copy")
    return out.value


def fma_rate(prec: str = "fp32") -> float:
    """Sustained non-packed FMA rate in flop per second ("fp32" or "fp64")."""
    if prec not in ("fp32", "fp64"):
        raise ValueError("fma_rate: fp32 or fp64")
    sink = torch.zeros(2, dtype=torch.float64, device=torch.cuda.current_device())
    out = C.c_double(0.0)
    _check(load().dirac_probe_fma(1 if prec == "fp64" else 0, sink.data_ptr(), C.byref(out), _stream()),
           "dirac_probe_fma")
    return out.value


def row_gather_rate(dims, site_bytes: int, src: torch.Tensor, dst: torch.Tensor, reps: int = 10,
                    nrows: int = 7) -> float:
    """Rate of the stencils' seven-row gather (nrows = 7) or of the row-by-row copy with the same loads
    (nrows = 1) on a (nx, ny, nz, nt) lattice of site_bytes-byte site blocks, in (one read + one write of the
    vector) bytes per second.  src and dst hold at least the vector each."""
    nx, ny, nz, nt = (int(d) for d in dims)
    need = nx * ny * nz * nt * int(site_bytes)
    for t, name in ((src, "src"), (dst, "dst")):
        if t.numel() * t.element_size() < need:
            raise ValueError(f"row_gather_rate: {name} holds fewer than {need} bytes")
    out = C.c_double(0.0)
    _check(load().dirac_probe_row_gather(_dev(src, "src"), _dev(dst, "dst"), nx, ny, nz, nt, int(site_bytes),
                                         int(nrows), reps, C.byref(out), _stream()), "dirac_probe_row_gather")
    return out.value
