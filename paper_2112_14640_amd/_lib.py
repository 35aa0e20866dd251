"""ctypes declarations of libdirac's C ABI (include/dirac.h).

The shared library is built in-tree by ``paper_2112_14640_amd.build`` and loaded
from this package directory.  There is no fallback: if it is missing, every
call raises.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdirac.so")

OK, NOT_CONVERGED, EINVAL, EUNSUPPORTED, EHIP, EWORKSPACE, ENONFINITE = 0, 1, -1, -2, -3, -4, -5

WILSON, BRILLOUIN, STAGGERED, WILSON_LAPLACE, BRILLOUIN_LAPLACE = 0, 1, 2, 3, 4
FP64, FP32, BF16 = 0, 1, 2


class Dims(C.Structure):
    _fields_ = [("n", C.c_int32 * 4), ("antiperiodic_t", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [
        ("iters", C.c_int),
        ("outer_iters", C.c_int),
        ("reason", C.c_int),
        ("true_relres", C.POINTER(C.c_double)),
        ("alpha", C.POINTER(C.c_double)),
        ("beta", C.POINTER(C.c_double)),
        ("hist_cap", C.c_int),
        ("hist_len", C.c_int),
    ]


class SolveOpts(C.Structure):
    _fields_ = [
        ("recompute_every", C.c_int),
        ("drift", C.c_double),
        ("mixed_scheme", C.c_int),
        ("delta", C.c_double),
        ("max_outer", C.c_int),
        ("clover_hi", C.c_void_p),
        ("clover_lo", C.c_void_p),
    ]


_vp = C.c_void_p
_i = C.c_int
_d = C.c_double
_i64 = C.c_int64
_sz = C.c_size_t
_dims = C.POINTER(Dims)

SIGNATURES = {
    "dirac_apply": (_i, [_i, _i, _vp, _vp, _vp, _d, _i, _i, _dims, _vp]),
    "dirac_apply_dagger": (_i, [_i, _i, _vp, _vp, _vp, _d, _i, _i, _dims, _vp]),
    "dirac_apply_normal": (_i, [_i, _i, _vp, _vp, _vp, _vp, _d, _i, _i, _dims, _vp]),
    "dirac_apply_clover": (_i, [_i, _i, _vp, _vp, _vp, _vp, _d, _i, _i, _dims, _vp]),
    "dirac_apply_clover_dagger": (_i, [_i, _i, _vp, _vp, _vp, _vp, _d, _i, _i, _dims, _vp]),
    "dirac_clover_field_bytes": (_sz, [_i, _i, _dims]),
    "dirac_clover_field": (_i, [_i, _vp, _d, _vp, _i, _dims, _vp]),
    "dirac_brillouin_links": (_i, [_i, _vp, _vp, _i, _dims, _vp]),
    "dirac_force": (_i, [_i, _vp, _vp, _vp, _vp, _d, _i, _i, _dims, _vp]),
    "dirac_project_su": (_i, [_vp, _vp, _vp, _i, _i64, _vp]),
    "dirac_stout_smear": (_i, [_vp, _vp, _d, _i, _dims, _vp]),
    "dirac_stout_backward": (_i, [_vp, _vp, _vp, _d, _i, _dims, _vp]),
    "dirac_brillouin_links_backward": (_i, [_vp, _vp, _vp, _i, _dims, _vp]),
    "dirac_blas_workspace_bytes": (_sz, [_i]),
    "dirac_norm2": (_i, [_i, _vp, _i64, _i, _vp, _vp, _sz, _vp]),
    "dirac_dot": (_i, [_i, _vp, _i, _vp, _i64, _i, _vp, _vp, _sz, _vp]),
    "dirac_dot_noalloc": (_i, [_i, _vp, _i, _vp, _i64, _i, _vp, _vp]),
    "dirac_caxpy": (_i, [_i, _vp, _i, _vp, _vp, _i64, _i, _vp]),
    "dirac_cxpay": (_i, [_i, _vp, _i, _vp, _vp, _i64, _i, _vp]),
    "dirac_cast": (_i, [_i, _vp, _i, _vp, _i64, _vp]),
    "dirac_gamma5": (_i, [_i, _i, _vp, _vp, _i, _i, _dims, _vp]),
    "dirac_solver_workspace_bytes": (_sz, [_i, _i, _i, _i, _i, _i, _dims]),
    "cg_solve": (_i, [_i, _i, _i, _vp, _vp, _vp, _vp, _d, _i, _i, _dims, _d, _i, _vp, _sz, C.POINTER(SolveInfo),
                      C.POINTER(SolveOpts), _vp]),
    "bicgstab_solve": (_i, [_i, _i, _i, _vp, _vp, _vp, _vp, _d, _i, _i, _dims, _d, _i, _vp, _sz,
                            C.POINTER(SolveInfo), C.POINTER(SolveOpts), _vp]),
    "dirac_set_launch_shape": (_i, [_i, _i, _i, _i]),
    "dirac_flops_per_site": (_d, [_i, _i]),
    "dirac_error_string": (C.c_char_p, [_i]),
    "dirac_last_error": (C.c_char_p, []),
    "dirac_version": (C.c_char_p, []),
}

_lib = None


class DiracError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        msg = lib.dirac_error_string(status).decode()
        detail = lib.dirac_last_error().decode()
        super().__init__(f"{where}: {msg} ({status}): {detail}")
        self.status = status


def load():
    """Load libdirac.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with `python -m paper_2112_14640_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, where: str, allow_not_converged: bool = False) -> int:
    if status == OK or (allow_not_converged and status == NOT_CONVERGED):
        return status
    raise DiracError(status, where)
