"""Torch-facing binding of libdirac: argument marshalling only.

Every operation runs in the HIP library on the tensors' device and on torch's
current stream; this module checks shapes, dtypes and devices, allocates
outputs with torch, and forwards device pointers.  There is no CPU path.

Layouts (x fastest among sites, right-hand-side index fastest inside a site):

* gauge ``U``: (Nt, Nz, Ny, Nx, 4, Nc, Nc) complex
* Brillouin links ``W``: (Nt, Nz, Ny, Nx, 40, Nc, Nc) complex (from ``brillouin_links``)
* clover field: (Nt, Nz, Ny, Nx, 8 Nc^2) real (from ``clover_field``), float64 or float32
* Wilson/Brillouin vectors (also for the two Laplacians): (Nt, Nz, Ny, Nx, Nc, 4, Nv)
* staggered vectors: (Nt, Nz, Ny, Nx, Nc, Nv)

Operators: "wilson", "brillouin", "staggered", and the hermitian Laplacians "wilson_laplace"
(gauge U) and "brillouin_laplace" (gauge W).

Precision follows the vector dtype: complex128 -> FP64 (complex128 gauge),
complex64 -> FP32 (complex64 gauge), bfloat16 with a trailing (re, im) axis of
size 2 -> BF16 storage with FP32 arithmetic (complex64 gauge).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L

OPS = {"wilson": L.WILSON, "brillouin": L.BRILLOUIN, "staggered": L.STAGGERED, "wilson_laplace": L.WILSON_LAPLACE,
       "brillouin_laplace": L.BRILLOUIN_LAPLACE}
PREC_NAMES = {L.FP64: "fp64", L.FP32: "fp32", L.BF16: "bf16"}
_PRECS = {v: k for k, v in PREC_NAMES.items()}


def _op(op) -> int:
    if isinstance(op, int):
        return op
    return OPS[op]


def vector_prec(x: torch.Tensor) -> int:
    if x.dtype == torch.complex128:
        return L.FP64
    if x.dtype == torch.complex64:
        return L.FP32
    if x.dtype == torch.bfloat16 and x.shape[-1] == 2:
        return L.BF16
    raise TypeError(f"unsupported vector dtype {x.dtype} (shape {tuple(x.shape)})")


def _gauge_dtype(prec: int):
    return torch.complex128 if prec == L.FP64 else torch.complex64


def _cshape(x: torch.Tensor, prec: int):
    """Logical complex shape of a vector tensor (drops the BF16 (re, im) axis)."""
    return tuple(x.shape[:-1]) if prec == L.BF16 else tuple(x.shape)


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _require(t: torch.Tensor, name: str, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (libdirac has no CPU path)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")


def _require_like(t: torch.Tensor, name: str, ref: torch.Tensor):
    """t must be a contiguous tensor on ref's device with ref's exact shape and dtype (an output or
    scratch buffer the library writes as many bytes into as ref holds)."""
    _require(t, name, ref.device)
    if tuple(t.shape) != tuple(ref.shape):
        raise ValueError(f"{name} shape {tuple(t.shape)} != {tuple(ref.shape)}")
    if t.dtype != ref.dtype:
        raise TypeError(f"{name} dtype {t.dtype} != {ref.dtype}")


@dataclass
class Geometry:
    op: int
    prec: int
    nc: int
    nv: int
    dims: tuple  # (Nx, Ny, Nz, Nt)
    antiperiodic_t: bool

    def cdims(self) -> L.Dims:
        d = L.Dims()
        for i, n in enumerate(self.dims):
            d.n[i] = n
        d.antiperiodic_t = 1 if self.antiperiodic_t else 0
        return d

    @property
    def volume(self) -> int:
        nx, ny, nz, nt = self.dims
        return nx * ny * nz * nt

    @property
    def nrows(self) -> int:
        return self.volume * self.nc * (1 if self.op == L.STAGGERED else 4)


def geometry(op, u: torch.Tensor, antiperiodic_t=True) -> Geometry:
    op = _op(op)
    prec = vector_prec(u)
    s = _cshape(u, prec)
    want = 6 if op == L.STAGGERED else 7
    if len(s) != want or (op != L.STAGGERED and s[5] != 4):
        kind = "(Nt,Nz,Ny,Nx,Nc,Nv)" if op == L.STAGGERED else "(Nt,Nz,Ny,Nx,Nc,4,Nv)"
        raise ValueError(f"vector shape {s} does not match {kind}")
    nt, nz, ny, nx, nc = s[:5]
    return Geometry(op, prec, nc, s[-1], (nx, ny, nz, nt), antiperiodic_t)


def _check_gauge(g: Geometry, gauge: torch.Tensor, name="gauge", device=None):
    _require(gauge, name, device)
    nx, ny, nz, nt = g.dims
    dirs = 40 if g.op in (L.BRILLOUIN, L.BRILLOUIN_LAPLACE) else 4
    want = (nt, nz, ny, nx, dirs, g.nc, g.nc)
    if tuple(gauge.shape) != want:
        raise ValueError(f"{name} shape {tuple(gauge.shape)} != {want}")
    if gauge.dtype != _gauge_dtype(g.prec):
        raise TypeError(f"{name} dtype {gauge.dtype} != {_gauge_dtype(g.prec)} for {PREC_NAMES[g.prec]} vectors")


def _clover_dtype(prec: int):
    return torch.float64 if prec == L.FP64 else torch.float32


def _check_clover(g: Geometry, clover: torch.Tensor, name="clover", device=None):
    _require(clover, name, device)
    if g.op not in (L.WILSON, L.BRILLOUIN):
        raise ValueError("the clover term belongs to the Wilson and Brillouin operators")
    nx, ny, nz, nt = g.dims
    want = (nt, nz, ny, nx, 8 * g.nc * g.nc)
    if tuple(clover.shape) != want:
        raise ValueError(f"{name} shape {tuple(clover.shape)} != {want}")
    if clover.dtype != _clover_dtype(g.prec):
        raise TypeError(f"{name} dtype {clover.dtype} != {_clover_dtype(g.prec)} for {PREC_NAMES[g.prec]} vectors")


def _apply(fn, op, gauge, u, mass, antiperiodic_t, out, clover=None):
    _require(u, "u")
    g = geometry(op, u, antiperiodic_t)
    _check_gauge(g, gauge, device=u.device)
    if out is None:
        out = torch.empty_like(u)
    else:
        _require_like(out, "out", u)
    lib = L.load()
    d = g.cdims()
    if clover is None:
        L.check(getattr(lib, fn)(g.op, g.prec, _ptr(gauge), _ptr(u), _ptr(out), float(mass), g.nc, g.nv, C.byref(d),
                                 _stream()), fn)
    else:
        _check_clover(g, clover, device=u.device)
        fn = fn.replace("dirac_apply", "dirac_apply_clover")
        L.check(getattr(lib, fn)(g.op, g.prec, _ptr(gauge), _ptr(clover), _ptr(u), _ptr(out), float(mass), g.nc,
                                 g.nv, C.byref(d), _stream()), fn)
    return out


def apply(op, gauge, u, mass, antiperiodic_t=True, out=None, clover=None):
    """v = D u for op in OPS (gauge = U, or W for the Brillouin operators); with ``clover`` (Wilson,
    Brillouin) v = (D + C) u."""
    return _apply("dirac_apply", op, gauge, u, mass, antiperiodic_t, out, clover)


def apply_dagger(op, gauge, u, mass, antiperiodic_t=True, out=None, clover=None):
    """v = D^dagger u (with ``clover``: (D + C)^dagger u = D^dagger u + C u)."""
    return _apply("dirac_apply_dagger", op, gauge, u, mass, antiperiodic_t, out, clover)


def clover_field(U, csw, antiperiodic_t=True, out=None):
    """Packed clover field of C = -(c_SW/2) sum sigma F (Eq. def_clov) from U: (Nt,Nz,Ny,Nx,8 Nc^2) real,
    float64 for complex128 links and float32 for complex64 links."""
    _require(U, "U")
    if U.dim() != 7 or U.shape[4] != 4 or U.shape[5] != U.shape[6]:
        raise ValueError(f"U shape {tuple(U.shape)} is not (Nt,Nz,Ny,Nx,4,Nc,Nc)")
    prec = {torch.complex128: L.FP64, torch.complex64: L.FP32}.get(U.dtype)
    if prec is None:
        raise TypeError("U must be complex128 or complex64")
    nt, nz, ny, nx, _, nc, _ = U.shape
    want = (nt, nz, ny, nx, 8 * nc * nc)
    if out is None:
        out = torch.empty(want, dtype=_clover_dtype(prec), device=U.device)
    else:
        _require(out, "out", U.device)
        if tuple(out.shape) != want or out.dtype != _clover_dtype(prec):
            raise ValueError(f"out must be a {want} tensor of {_clover_dtype(prec)}")
    d = L.Dims()
    for i, n in enumerate((nx, ny, nz, nt)):
        d.n[i] = n
    d.antiperiodic_t = 1 if antiperiodic_t else 0
    L.check(L.load().dirac_clover_field(prec, _ptr(U), float(csw), _ptr(out), nc, C.byref(d), _stream()),
            "dirac_clover_field")
    return out


def apply_normal(op, gauge, u, mass, antiperiodic_t=True, out=None, tmp=None):
    """v = D^dagger D u (through a scratch vector)."""
    _require(u, "u")
    g = geometry(op, u, antiperiodic_t)
    _check_gauge(g, gauge, device=u.device)
    out = torch.empty_like(u) if out is None else out
    tmp = torch.empty_like(u) if tmp is None else tmp
    _require_like(out, "out", u)
    _require_like(tmp, "tmp", u)
    d = g.cdims()
    L.check(L.load().dirac_apply_normal(g.op, g.prec, _ptr(gauge), _ptr(u), _ptr(out), _ptr(tmp), float(mass), g.nc,
                                        g.nv, C.byref(d), _stream()), "dirac_apply_normal")
    return out


def brillouin_links(U, antiperiodic_t=True, out=None):
    """Stored Brillouin links W (Nt,Nz,Ny,Nx,40,Nc,Nc) from U (same dtype; complex128 or complex64)."""
    _require(U, "U")
    if U.dim() != 7 or U.shape[4] != 4 or U.shape[5] != U.shape[6]:
        raise ValueError(f"U shape {tuple(U.shape)} is not (Nt,Nz,Ny,Nx,4,Nc,Nc)")
    prec = {torch.complex128: L.FP64, torch.complex64: L.FP32}.get(U.dtype)
    if prec is None:
        raise TypeError("U must be complex128 or complex64")
    nt, nz, ny, nx, _, nc, _ = U.shape
    if out is None:
        out = torch.empty((nt, nz, ny, nx, 40, nc, nc), dtype=U.dtype, device=U.device)
    else:
        _require(out, "out", U.device)
        if tuple(out.shape) != (nt, nz, ny, nx, 40, nc, nc) or out.dtype != U.dtype:
            raise ValueError("out must be a (Nt,Nz,Ny,Nx,40,Nc,Nc) tensor of U's dtype")
    d = L.Dims()
    for i, n in enumerate((nx, ny, nz, nt)):
        d.n[i] = n
    d.antiperiodic_t = 1 if antiperiodic_t else 0
    L.check(L.load().dirac_brillouin_links(prec, _ptr(U), _ptr(out), nc, C.byref(d), _stream()),
            "dirac_brillouin_links")
    return out


def _link_dims(U, dirs=4):
    """(Nx,Ny,Nz,Nt), Nc of a complex128 link field (Nt,Nz,Ny,Nx,dirs,Nc,Nc) on the GPU."""
    _require(U, "links")
    if U.dim() != 7 or U.shape[4] != dirs or U.shape[5] != U.shape[6]:
        raise ValueError(f"link shape {tuple(U.shape)} is not (Nt,Nz,Ny,Nx,{dirs},Nc,Nc)")
    if U.dtype != torch.complex128:
        raise TypeError("smearing and link gradients are FP64 (complex128)")
    nt, nz, ny, nx = U.shape[:4]
    d = L.Dims()
    for i, n in enumerate((nx, ny, nz, nt)):
        d.n[i] = n
    d.antiperiodic_t = 1
    return d, U.shape[-1]


def stout_step(U, rho, out=None):
    """One stout-smearing step (Sec. 2): V_mu(n) = exp(i Q_mu(n)) U_mu(n); FP64."""
    d, nc = _link_dims(U)
    out = torch.empty_like(U) if out is None else out
    _require_like(out, "out", U)
    L.check(L.load().dirac_stout_smear(_ptr(U), _ptr(out), float(rho), nc, C.byref(d), _stream()),
            "dirac_stout_smear")
    return out


def stout_smear(U, rho=0.12, steps=3):
    """``steps`` stout steps with parameter ``rho`` (the paper's defaults); FP64."""
    V = U
    for _ in range(steps):
        V = stout_step(V, rho)
    return V.clone() if steps == 0 else V


def stout_backward(U, gV, rho, out=None):
    """out += dL/dU for one stout step U -> V given gV = dL/dV (U is the step's input); FP64."""
    d, nc = _link_dims(U)
    _require_like(gV, "gV", U)
    out = torch.zeros_like(U) if out is None else out
    _require_like(out, "out", U)
    L.check(L.load().dirac_stout_backward(_ptr(U), _ptr(gV), _ptr(out), float(rho), nc, C.byref(d), _stream()),
            "dirac_stout_backward")
    return out


def brillouin_links_backward(V, gW, out=None):
    """out += dL/dV for W = brillouin_links(V) given gW = dL/dW (40 stored directions); FP64."""
    d, nc = _link_dims(V)
    _link_dims(gW, 40)
    if gW.shape[:4] != V.shape[:4] or gW.shape[-1] != nc or gW.device != V.device:
        raise ValueError("gW does not match V")
    out = torch.zeros_like(V) if out is None else out
    _require_like(out, "out", V)
    L.check(L.load().dirac_brillouin_links_backward(_ptr(V), _ptr(gW), _ptr(out), nc, C.byref(d), _stream()),
            "dirac_brillouin_links_backward")
    return out


def force(op, U, psi, chi, coeff=1.0, antiperiodic_t=True, out=None):
    """out += coeff * d Re(psi^dagger D chi) / dU (torch's complex-gradient convention); FP64.  For the
    Brillouin operator U is the stored-link array W and the gradient is with respect to W."""
    _require(psi, "psi")
    for t, n in ((U, "U"), (chi, "chi")):
        _require(t, n, psi.device)
    g = geometry(op, psi, antiperiodic_t)
    if g.prec != L.FP64 or chi.dtype != torch.complex128 or U.dtype != torch.complex128:
        raise TypeError("force is FP64 (complex128) only")
    if chi.shape != psi.shape:
        raise ValueError("psi and chi must have the same shape")
    _check_gauge(g, U, "U")
    out = torch.zeros_like(U) if out is None else out
    _require_like(out, "out", U)
    d = g.cdims()
    L.check(L.load().dirac_force(g.op, _ptr(U), _ptr(psi), _ptr(chi), _ptr(out), float(coeff), g.nc, g.nv,
                                 C.byref(d), _stream()), "dirac_force")
    return out


def project_su(U, g, out=None):
    """su(Nc) force (i/2)(U g^+ - g U^+) - trace/Nc, FP64."""
    _require(U, "U")
    _require(g, "g", U.device)
    if U.dtype != torch.complex128 or g.dtype != torch.complex128 or U.shape != g.shape:
        raise TypeError("U and g must be complex128 tensors of the same shape")
    if U.dim() < 2 or U.shape[-1] != U.shape[-2]:
        raise ValueError("U must end in a square (Nc, Nc) matrix axis")
    nc = U.shape[-1]
    out = torch.empty_like(U) if out is None else out
    _require_like(out, "out", U)
    L.check(L.load().dirac_project_su(_ptr(U), _ptr(g), _ptr(out), nc, U.numel() // (nc * nc), _stream()),
            "dirac_project_su")
    return out


# ---------------------------------------------------------------------------
# BLAS-1 (per right-hand side)
# ---------------------------------------------------------------------------
def _rows(x: torch.Tensor, prec: int):
    s = _cshape(x, prec)
    nv = s[-1]
    n = 1
    for k in s[:-1]:
        n *= k
    return n, nv


def _blas_ws(nv: int, device) -> torch.Tensor:
    nbytes = L.load().dirac_blas_workspace_bytes(nv)
    return torch.empty(nbytes // 8, dtype=torch.float64, device=device)


def norm2(x: torch.Tensor) -> torch.Tensor:
    """||x_i||^2 per RHS (float64 tensor of length Nv, on the device)."""
    _require(x, "x")
    p = vector_prec(x)
    nrows, nv = _rows(x, p)
    out = torch.empty(nv, dtype=torch.float64, device=x.device)
    ws = _blas_ws(nv, x.device)
    L.check(L.load().dirac_norm2(p, _ptr(x), nrows, nv, _ptr(out), _ptr(ws), ws.numel() * 8, _stream()), "norm2")
    return out


def dot(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """<x_i, y_i> = sum conj(x) y per RHS (complex128, length Nv)."""
    _require(x, "x")
    _require(y, "y", x.device)
    px, py = vector_prec(x), vector_prec(y)
    nrows, nv = _rows(x, px)
    if _rows(y, py) != (nrows, nv):
        raise ValueError("x and y differ in shape")
    out = torch.empty(2 * nv, dtype=torch.float64, device=x.device)
    ws = _blas_ws(nv, x.device)
    L.check(L.load().dirac_dot(px, _ptr(x), py, _ptr(y), nrows, nv, _ptr(out), _ptr(ws), ws.numel() * 8, _stream()),
            "dot")
    return torch.view_as_complex(out.view(nv, 2))


def _coef(a, nv, device):
    a = torch.as_tensor(a, dtype=torch.complex128, device=device).reshape(-1)
    if a.numel() == 1:
        a = a.expand(nv)
    if a.numel() != nv:
        raise ValueError("coefficient must be a scalar or have Nv entries")
    return torch.view_as_real(a.contiguous()).contiguous()


def caxpy(a, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """y_i += a_i x_i in place (the paper's "incr")."""
    _require(x, "x")
    _require(y, "y", x.device)
    px, py = vector_prec(x), vector_prec(y)
    nrows, nv = _rows(x, px)
    if _rows(y, py) != (nrows, nv):
        raise ValueError("x and y differ in shape")
    c = _coef(a, nv, x.device)
    L.check(L.load().dirac_caxpy(px, _ptr(x), py, _ptr(y), _ptr(c), nrows, nv, _stream()), "caxpy")
    return y


def cxpay(x: torch.Tensor, a, y: torch.Tensor) -> torch.Tensor:
    """y_i = x_i + a_i y_i in place (the paper's "anti")."""
    _require(x, "x")
    _require(y, "y", x.device)
    px, py = vector_prec(x), vector_prec(y)
    nrows, nv = _rows(x, px)
    if _rows(y, py) != (nrows, nv):
        raise ValueError("x and y differ in shape")
    c = _coef(a, nv, x.device)
    L.check(L.load().dirac_cxpay(px, _ptr(x), py, _ptr(y), _ptr(c), nrows, nv, _stream()), "cxpay")
    return y


def empty_vector(shape, prec: int, device) -> torch.Tensor:
    """Uninitialised vector of complex shape `shape` in precision `prec`."""
    if prec == L.FP64:
        return torch.empty(shape, dtype=torch.complex128, device=device)
    if prec == L.FP32:
        return torch.empty(shape, dtype=torch.complex64, device=device)
    return torch.empty(tuple(shape) + (2,), dtype=torch.bfloat16, device=device)


def cast(x: torch.Tensor, prec) -> torch.Tensor:
    """Convert a vector to another storage precision ("fp64", "fp32", "bf16"; BF16 rounds to nearest even)."""
    _require(x, "x")
    if isinstance(prec, str):
        prec = {"fp64": L.FP64, "fp32": L.FP32, "bf16": L.BF16}[prec]
    px = vector_prec(x)
    shape = _cshape(x, px)
    y = empty_vector(shape, prec, x.device)
    n = 1
    for k in shape:
        n *= k
    L.check(L.load().dirac_cast(px, _ptr(x), prec, _ptr(y), n, _stream()), "cast")
    return y


def gamma5(op, x: torch.Tensor, antiperiodic_t=True, out=None) -> torch.Tensor:
    """gamma_5 x (Wilson/Brillouin layout) or epsilon x (staggered layout)."""
    _require(x, "x")
    g = geometry(op, x, antiperiodic_t)
    out = torch.empty_like(x) if out is None else out
    _require_like(out, "out", x)
    d = g.cdims()
    L.check(L.load().dirac_gamma5(g.op, g.prec, _ptr(x), _ptr(out), g.nc, g.nv, C.byref(d), _stream()), "gamma5")
    return out


# ---------------------------------------------------------------------------
# Solvers
# ---------------------------------------------------------------------------
@dataclass
class SolveInfo:
    status: int
    iterations: int
    outer_iterations: int
    reason: str
    true_relres: list
    alphas: list
    betas: list


def _solve(fn, solver, op, gauge, b, mass, x0, tol, maxit, inner, gauge_lo, antiperiodic_t, history, opts,
           clover=None, clover_lo=None):
    _require(b, "b")
    g = geometry(op, b, antiperiodic_t)
    _check_gauge(g, gauge, device=b.device)
    outer = g.prec
    inner_p = outer if inner is None else {"fp64": L.FP64, "fp32": L.FP32, "bf16": L.BF16}[inner]
    if inner_p != outer:
        if gauge_lo is None:
            raise ValueError("mixed precision needs gauge_lo (complex64 links)")
        gl = Geometry(g.op, inner_p, g.nc, g.nv, g.dims, g.antiperiodic_t)
        _check_gauge(gl, gauge_lo, "gauge_lo", device=b.device)
    x = torch.zeros_like(b)
    if x0 is not None:
        if not isinstance(x0, torch.Tensor):
            raise TypeError("x0 must be a tensor")
        if x0.device != b.device or tuple(x0.shape) != tuple(b.shape) or x0.dtype != b.dtype:
            raise ValueError("x0 must match b in device, shape and dtype")
        x.copy_(x0)
    lib = L.load()
    d = g.cdims()
    nbytes = lib.dirac_solver_workspace_bytes(g.op, solver, outer, inner_p, g.nc, g.nv, C.byref(d))
    if nbytes == 0:
        raise ValueError("invalid solver configuration")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
    info = L.SolveInfo()
    relres = (C.c_double * g.nv)()
    info.true_relres = relres
    cap = maxit if history else 0
    ha = (C.c_double * max(1, cap * g.nv))()
    hb = (C.c_double * max(1, cap * g.nv))()
    if history:
        info.alpha = ha
        info.beta = hb
        info.hist_cap = cap
    o = L.SolveOpts()
    for k, v in (opts or {}).items():
        setattr(o, k, v)
    if clover is not None:
        _check_clover(g, clover, device=b.device)
        o.clover_hi = _ptr(clover)
        if inner_p != outer:
            if clover_lo is None:
                raise ValueError("a mixed solve with a clover term needs clover_lo (float32)")
            _check_clover(Geometry(g.op, inner_p, g.nc, g.nv, g.dims, g.antiperiodic_t), clover_lo, "clover_lo",
                          b.device)
            o.clover_lo = _ptr(clover_lo)
    status = getattr(lib, fn)(g.op, outer, inner_p, _ptr(gauge), _ptr(gauge_lo) if gauge_lo is not None else None,
                              _ptr(b), _ptr(x), float(mass), g.nc, g.nv, C.byref(d), float(tol), int(maxit), _ptr(ws),
                              nbytes, C.byref(info), C.byref(o), _stream())
    L.check(status, fn, allow_not_converged=True)
    n = info.hist_len
    alphas = [[ha[k * g.nv + i] for i in range(g.nv)] for k in range(n)] if history else []
    betas = [[hb[k * g.nv + i] for i in range(g.nv)] for k in range(n)] if history else []
    reason = {0: "converged", 1: "stagnated", 2: "maxit"}[info.reason]
    return x, SolveInfo(status, info.iters, info.outer_iters, reason, list(relres), alphas, betas)


def cg(op, gauge, b, mass, x0=None, tol=1e-10, maxit=1000, inner=None, gauge_lo=None, antiperiodic_t=True,
       history=False, opts=None, clover=None, clover_lo=None):
    """Solve D^dagger D x = b by CG (N_v RHS in lock-step; D x = b for the hermitian Laplacians).
    inner="fp32"/"bf16" for mixed precision; clover (and clover_lo when mixed) for D + C."""
    return _solve("cg_solve", 0, op, gauge, b, mass, x0, tol, maxit, inner, gauge_lo, antiperiodic_t, history, opts,
                  clover, clover_lo)


def bicgstab(op, gauge, b, mass, x0=None, tol=1e-10, maxit=1000, inner=None, gauge_lo=None, antiperiodic_t=True,
             opts=None, clover=None, clover_lo=None):
    """Solve D x = b by BiCGstab (Wilson, Brillouin).  inner="fp32"/"bf16" for defect-correction mixed precision."""
    return _solve("bicgstab_solve", 1, op, gauge, b, mass, x0, tol, maxit, inner, gauge_lo, antiperiodic_t, False,
                  opts, clover, clover_lo)


def flops_per_site(op, nc: int) -> float:
    """App. E flop count per site and RHS of one apply."""
    return L.load().dirac_flops_per_site(_op(op), nc)


def set_launch_shape(op, prec, rb: int = 0, variant: int = 0):
    """Launch-shape knob of the stencil kernels: RHS columns per thread (0 = automatic) and variant
    (0 = automatic, 1 = direct global loads, 4 = row tiles staged in LDS; see include/dirac.h)."""
    if isinstance(prec, str):
        prec = {"fp64": L.FP64, "fp32": L.FP32, "bf16": L.BF16}[prec]
    L.check(L.load().dirac_set_launch_shape(_op(op), prec, rb, variant), "set_launch_shape")
