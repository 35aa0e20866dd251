"""Helpers shared by the GPU parity tests (inputs on the host, results compared on the host)."""
import numpy as np
import torch

DEV = "cuda:0"


def to_dev(a: np.ndarray, dtype=torch.complex128) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dtype)


def to_bf16_pairs(a: np.ndarray) -> torch.Tensor:
    """complex host array -> device bfloat16 tensor with a trailing (re, im) axis (RNE from FP32)."""
    t = torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64)))
    return torch.view_as_real(t).to(torch.bfloat16).contiguous().to(DEV)


def bf16_pairs_to_host(t: torch.Tensor) -> np.ndarray:
    f = t.float().cpu().numpy()
    return f[..., 0] + 1j * f[..., 1]


def host(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy()


def round_c64(a: np.ndarray) -> np.ndarray:
    """The complex128 value of a's complex64 rounding (the oracle's input for FP32 parity)."""
    return a.astype(np.complex64).astype(np.complex128)


def round_bf16(a: np.ndarray) -> np.ndarray:
    """The value of a after FP32 then bfloat16 round-to-nearest-even rounding, as complex128."""
    t = torch.view_as_real(torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))))
    b = t.to(torch.bfloat16).double().numpy()
    return b[..., 0] + 1j * b[..., 1]


def col_rel_err(v: np.ndarray, ref: np.ndarray) -> float:
    """max over RHS columns of ||v_i - ref_i|| / ||ref_i|| (RHS = last axis)."""
    a = v.reshape(-1, v.shape[-1])
    b = ref.reshape(-1, ref.shape[-1])
    num = np.linalg.norm(a - b, axis=0)
    den = np.linalg.norm(b, axis=0)
    return float(np.max(num / np.maximum(den, 1e-300)))


def elem_rel_err(v: np.ndarray, ref: np.ndarray) -> float:
    """max |v - ref| over every element / max |ref|: a localized error is not diluted by the column norm."""
    return float(np.max(np.abs(v - ref)) / max(float(np.max(np.abs(ref))), 1e-300))


def parity(v: np.ndarray, ref: np.ndarray, tol: float, what=""):
    """Both bars: worst RHS column 2-norm error and element-wise max error, each relative, below tol."""
    ce, ee = col_rel_err(v, ref), elem_rel_err(v, ref)
    assert ce < tol and ee < tol, (what, "column", ce, "element", ee, "tol", tol)
    return ce, ee


def unpack_clover(packed: np.ndarray, nc: int) -> np.ndarray:
    """Packed clover blocks (..., 8 nc^2) -> (..., 4 nc, 4 nc) matrices indexed (colour, spin) as the
    vector layout: block h holds spins 2h, 2h+1; within a block component i is spin 2h + i // nc, colour
    i % nc; N = 2 nc diagonal reals, then (re, im) of (i, j), i < j, row by row."""
    n = 2 * nc
    lead = packed.shape[:-1]
    out = np.zeros(lead + (4 * nc, 4 * nc), dtype=np.complex128)
    for h in range(2):
        b = packed[..., h * n * n:(h + 1) * n * n].astype(np.float64)
        blk = np.zeros(lead + (n, n), dtype=np.complex128)
        for i in range(n):
            blk[..., i, i] = b[..., i]
        e = n
        for i in range(n):
            for j in range(i + 1, n):
                blk[..., i, j] = b[..., e] + 1j * b[..., e + 1]
                blk[..., j, i] = b[..., e] - 1j * b[..., e + 1]
                e += 2
        idx = [(i % nc) * 4 + 2 * h + i // nc for i in range(n)]
        for i in range(n):
            for j in range(n):
                out[..., idx[i], idx[j]] = blk[..., i, j]
    return out


def sample_sites(dims, count, seed=123, include_boundary=True):
    """Random site coordinates (x,y,z,t), plus sites on the t = 0 and t = Nt-1 slices."""
    rng = np.random.default_rng(seed)
    nx, ny, nz, nt = dims
    pts = np.stack([rng.integers(0, n, count) for n in (nx, ny, nz, nt)], axis=1)
    if include_boundary:
        k = max(count // 8, 8)
        b0 = np.stack([rng.integers(0, n, k) for n in (nx, ny, nz)] + [np.zeros(k, int)], axis=1)
        b1 = np.stack([rng.integers(0, n, k) for n in (nx, ny, nz)] + [np.full(k, nt - 1)], axis=1)
        corner = np.array([[0, 0, 0, 0], [nx - 1, ny - 1, nz - 1, nt - 1], [nx - 1, 0, nz - 1, 0]])
        pts = np.concatenate([pts, b0, b1, corner])
    return pts


def at_sites(field: np.ndarray, sites: np.ndarray) -> np.ndarray:
    """field[t, z, y, x, ...] gathered at (x, y, z, t) coordinates."""
    return field[sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0]]
