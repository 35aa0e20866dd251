"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the bench.

This module draws random numbers and shapes them into gauge links, source
vectors and gauge transformations.  It holds none of the Dirac-operator
arithmetic: no stencil, no gamma matrix, no solver.  Both the oracle and the
HIP path consume its arrays as plain data.

Conventions (host arrays, numpy complex128 unless a dtype is requested):

* gauge field ``U``: shape (Nt, Nz, Ny, Nx, 4, Nc, Nc); ``U[t,z,y,x,mu,a,b]`` is
  the row-a, column-b entry of the link U_mu(n) that transports from n+mu to n
  (mu = 0,1,2,3 for x,y,z,t).
* Wilson/Brillouin vector: shape (Nt, Nz, Ny, Nx, Nc, 4, Nv) (right-hand-side
  index fastest).
* staggered vector: shape (Nt, Nz, Ny, Nx, Nc, Nv).

Random draws happen in C order of the requested shape, links first, then
sources, each complex number as (g1 + i g2)/sqrt(2) with g1, g2 standard
normal draws (all g1 of the array first, then all g2).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "complex_gaussian",
    "haar_su_n",
    "near_identity_su_n",
    "gauge_field",
    "wilson_vector",
    "staggered_vector",
    "gauge_transform",
    "su_n_directions",
    "config",
]


def complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    """Complex normal CN(0,1): (g1 + i g2)/sqrt(2), unit variance per complex entry."""
    g1 = rng.standard_normal(shape)
    g2 = rng.standard_normal(shape)
    return (g1 + 1j * g2) / np.sqrt(2.0)


def haar_su_n(rng: np.random.Generator, shape, nc: int) -> np.ndarray:
    """Haar-distributed SU(nc) matrices by the QR method (Mezzadri 2007).

    Z complex Gaussian, Z = QR, Q <- Q diag(R_ii/|R_ii|) (Haar on U(nc)), then the
    determinant phase is removed by dividing by det^(1/nc) on the principal branch.
    """
    z = complex_gaussian(rng, tuple(shape) + (nc, nc))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / nc))[..., None, None]
    return q


def near_identity_su_n(rng: np.random.Generator, shape, nc: int, spread: float) -> np.ndarray:
    """U = exp(i * spread * H), H a random traceless hermitian Gaussian matrix.

    A_ij = CN(0,1), H = (A + A^dagger)/2 with its trace removed; the exponential
    is taken through the eigendecomposition of H.
    """
    a = complex_gaussian(rng, tuple(shape) + (nc, nc))
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / nc
    h = h - tr[..., None, None] * np.eye(nc)
    w, v = np.linalg.eigh(h)
    ph = np.exp(1j * spread * w)
    return (v * ph[..., None, :]) @ np.conj(np.swapaxes(v, -1, -2))


def gauge_field(rng: np.random.Generator, dims, nc: int, kind: str = "haar", spread: float = 0.3) -> np.ndarray:
    """Gauge field of shape (Nt,Nz,Ny,Nx,4,nc,nc); dims = (Nx,Ny,Nz,Nt).

    kind: "haar" (Haar SU(nc)), "near" (exp(i spread H)), "unit" (free field).
    """
    nx, ny, nz, nt = dims
    shape = (nt, nz, ny, nx, 4)
    if kind == "haar":
        return haar_su_n(rng, shape, nc)
    if kind == "near":
        return near_identity_su_n(rng, shape, nc, spread)
    if kind == "unit":
        return np.broadcast_to(np.eye(nc, dtype=np.complex128), shape + (nc, nc)).copy()
    raise ValueError(f"unknown gauge kind {kind!r}")


def wilson_vector(rng: np.random.Generator, dims, nc: int, nv: int) -> np.ndarray:
    """Complex Gaussian Wilson-type multi-RHS vector (Nt,Nz,Ny,Nx,nc,4,nv)."""
    nx, ny, nz, nt = dims
    return complex_gaussian(rng, (nt, nz, ny, nx, nc, 4, nv))


def staggered_vector(rng: np.random.Generator, dims, nc: int, nv: int) -> np.ndarray:
    """Complex Gaussian staggered multi-RHS vector (Nt,Nz,Ny,Nx,nc,nv)."""
    nx, ny, nz, nt = dims
    return complex_gaussian(rng, (nt, nz, ny, nx, nc, nv))


def gauge_transform(rng: np.random.Generator, dims, nc: int) -> np.ndarray:
    """One Haar SU(nc) matrix per site, shape (Nt,Nz,Ny,Nx,nc,nc)."""
    nx, ny, nz, nt = dims
    return haar_su_n(rng, (nt, nz, ny, nx), nc)


def su_n_directions(rng: np.random.Generator, dims, nc: int, count: int) -> np.ndarray:
    """`count` full-field traceless hermitian perturbation directions H_mu(n).

    Shape (count, Nt,Nz,Ny,Nx,4,nc,nc); each H drawn as in near_identity_su_n,
    without any global normalisation.
    """
    nx, ny, nz, nt = dims
    a = complex_gaussian(rng, (count, nt, nz, ny, nx, 4, nc, nc))
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / nc
    return h - tr[..., None, None] * np.eye(nc)


def config(name: str):
    """Named synthetic workloads (lattice, colours, RHS, mass, link recipe, seed).

    Returns a dict; the shapes and recipes follow the benchmark configurations
    of the Dirac-apply study (Wilson/Brillouin/staggered at N_v = 12, etc.).
    """
    table = {
        # Wilson 4^4, Nv=1, FP64, Haar links, m=0.1: dense brute-force check
        "wilson_4x4_dense": dict(dims=(4, 4, 4, 4), nc=3, nv=1, mass=0.1, links="haar", spread=None, seed=0),
        # all three operators at 16^3x32, Nv=12, FP32, near-identity links s=0.3, m=0.05
        "apply_16x32": dict(dims=(16, 16, 16, 32), nc=3, nv=12, mass=0.05, links="near", spread=0.3, seed=0),
        # mixed-precision CG on D_W^dag D_W at 32^3x64, Nv=12, s=0.5, m=0.01
        "cg_32x64": dict(dims=(32, 32, 32, 64), nc=3, nv=12, mass=0.01, links="near", spread=0.5, seed=0),
        # differentiation through a solve at 24^3x48, Nv=4, FP64
        "grad_24x48": dict(dims=(24, 24, 24, 48), nc=3, nv=4, mass=0.05, links="near", spread=0.3, seed=0),
        # large-volume Brillouin / staggered at 48^3x96, Nv=12, Haar links
        "apply_48x96": dict(dims=(48, 48, 48, 96), nc=3, nv=12, mass=0.05, links="haar", spread=None, seed=0),
    }
    return dict(table[name])


# ---------------------------------------------------------------------------
# Device-side generators (torch) for lattices too large to draw on the host.
# Same recipes as above, drawn from a seeded torch.Generator on the target device;
# the random streams differ from the NumPy ones, so these feed benchmarks, not the
# oracle comparisons.
# ---------------------------------------------------------------------------
def complex_gaussian_t(gen, shape, device, dtype=None):
    import torch

    dtype = dtype or torch.complex128
    real = torch.float64 if dtype == torch.complex128 else torch.float32
    g = torch.randn(tuple(shape) + (2,), generator=gen, device=device, dtype=real)
    return torch.view_as_complex(g / 2 ** 0.5).to(dtype)


def haar_su_n_t(gen, shape, nc, device, dtype=None):
    """Haar SU(nc): Gram-Schmidt on the columns of a complex Gaussian matrix (the QR method with a
    positive diagonal of R), then the determinant phase removed by det^(1/nc)."""
    import torch

    z = complex_gaussian_t(gen, tuple(shape) + (nc, nc), device, torch.complex128)
    cols = []
    for j in range(nc):
        v = z[..., :, j]
        for q in cols:
            v = v - (torch.conj(q) * v).sum(-1, keepdim=True) * q
        v = v / torch.linalg.vector_norm(v, dim=-1, keepdim=True)
        cols.append(v)
    q = torch.stack(cols, dim=-1)
    det = _det_small(q)
    q = q / (det ** (1.0 / nc))[..., None, None]
    return q.to(dtype or torch.complex128).contiguous()


def _det_small(m):
    """Determinant of (..., n, n) matrices by cofactor expansion along the first row (n <= 4)."""
    n = m.shape[-1]
    if n == 1:
        return m[..., 0, 0]
    det = 0
    for j in range(n):
        minor = m[..., 1:, [k for k in range(n) if k != j]]
        det = det + (-1) ** j * m[..., 0, j] * _det_small(minor)
    return det


def near_identity_su_n_t(gen, shape, nc, spread, device, dtype=None):
    """exp(i spread H), H traceless hermitian Gaussian (as near_identity_su_n); the exponential by a
    Taylor series after scaling by 2^-6 and six squarings (converged to double precision)."""
    import torch

    a = complex_gaussian_t(gen, tuple(shape) + (nc, nc), device, torch.complex128)
    h = 0.5 * (a + torch.conj(a.transpose(-1, -2)))
    tr = torch.diagonal(h, dim1=-2, dim2=-1).real.sum(-1) / nc
    h = h - tr[..., None, None] * torch.eye(nc, dtype=h.dtype, device=device)
    x = (1j * spread / 64.0) * h
    eye = torch.eye(nc, dtype=h.dtype, device=device).expand_as(x)
    term = eye.clone()
    u = eye.clone()
    for k in range(1, 16):
        term = torch.matmul(term, x.contiguous()) / k
        u = u + term
    for _ in range(6):
        u = torch.matmul(u, u.contiguous())
    return u.to(dtype or torch.complex128).contiguous()
