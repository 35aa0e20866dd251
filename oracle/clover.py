"""Clover term C = -(c_SW/2) sum_{mu<nu} sigma_{mu nu} F_{mu nu}(n) (Sec. 4, Eq. def_clov).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Field strength.  The paper names the clover-leaf field strength F_{mu nu}(n),
hermitian in colour space and built from the (possibly smeared) links, without
printing its formula.  Reading used here (the standard clover leaf):

    Q_{mu nu}(n) = sum of the four plaquettes of the (mu, nu) plane that start
                   and end at n, each run in the same sense (first mu, then nu):
        U_mu(n)         U_nu(n+mu)       U_mu(n+nu)^+     U_nu(n)^+
        U_nu(n)         U_mu(n+nu-mu)^+  U_nu(n-mu)^+     U_mu(n-mu)
        U_mu(n-mu)^+    U_nu(n-mu-nu)^+  U_mu(n-mu-nu)    U_nu(n-nu)
        U_nu(n-nu)^+    U_mu(n-nu)       U_nu(n-nu+mu)    U_mu(n)^+
    F_{mu nu}(n)  = (Q - Q^+) / (8 i), minus its trace / N_c,

the traceless hermitian matrix (an element of su(N_c), like the continuum field
strength).  Links are periodic in every direction.  The six planes are stored
in the paper's order (1,2), (1,3), (1,4), (2,3), (2,4), (3,4) (Sec. 4), i.e.
(mu, nu) = (0,1), (0,2), (0,3), (1,2), (1,3), (2,3) with 0..3 = x, y, z, t.

Apply.  sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] is formed from the App. A
gamma matrices; C acts on the (colour, spin) indices of each site and as the
identity on the right-hand sides.  D + C and (D + C)^+ = D^+ + C (C is
hermitian) give the clover-improved Wilson and Brillouin operators of
Eqs. def_wils and def_bril.
"""
from __future__ import annotations

import numpy as np

from .gamma import sigma_munu

PLANES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def _shift(f, mu, s):
    """g(n) = f(n + s * mu_hat) on a field indexed [t, z, y, x, ...] (periodic)."""
    return np.roll(f, -s, axis=3 - mu)


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def clover_leaves(U, mu, nu):
    """Q_{mu nu}(n): the sum of the four plaquette leaves at every site, (Nt,Nz,Ny,Nx,Nc,Nc)."""
    Um = U[..., mu, :, :]
    Un = U[..., nu, :, :]
    s = _shift
    leaf1 = Um @ s(Un, mu, 1) @ _dag(s(Um, nu, 1)) @ _dag(Un)
    leaf2 = Un @ _dag(s(s(Um, nu, 1), mu, -1)) @ _dag(s(Un, mu, -1)) @ s(Um, mu, -1)
    leaf3 = _dag(s(Um, mu, -1)) @ _dag(s(s(Un, mu, -1), nu, -1)) @ s(s(Um, mu, -1), nu, -1) @ s(Un, nu, -1)
    leaf4 = _dag(s(Un, nu, -1)) @ s(Um, nu, -1) @ s(s(Un, nu, -1), mu, 1) @ _dag(Um)
    return leaf1 + leaf2 + leaf3 + leaf4


def field_strength(U):
    """F_{mu nu}(n) for the six planes, shape (Nt,Nz,Ny,Nx,6,Nc,Nc) (module docstring)."""
    nc = U.shape[-1]
    out = []
    for mu, nu in PLANES:
        q = clover_leaves(U, mu, nu)
        f = (q - _dag(q)) / 8j
        tr = np.trace(f, axis1=-2, axis2=-1) / nc
        out.append(f - tr[..., None, None] * np.eye(nc))
    return np.stack(out, axis=-3)


def clover_apply(F, psi, csw, sites=None):
    """(C psi)(n) = -(c_SW/2) sum_{mu<nu} [sigma_{mu nu} (x) F_{mu nu}(n)] psi(n).

    F: (Nt,Nz,Ny,Nx,6,Nc,Nc); psi: (Nt,Nz,Ny,Nx,Nc,4,Nv).  With ``sites`` only those
    outputs, shape (S,Nc,4,Nv).
    """
    if sites is not None:
        sites = np.asarray(sites)
        F = F[sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0]]
        psi = psi[sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0]]
    out = np.zeros(psi.shape, dtype=np.complex128)
    for p, (mu, nu) in enumerate(PLANES):
        sig = sigma_munu(mu, nu)
        out = out + np.einsum("st,...ab,...btr->...asr", sig, F[..., p, :, :], psi)
    return -0.5 * csw * out


def clover_site_matrix(F_site, csw):
    """The 4 Nc x 4 Nc matrix of C at one site, index (colour, spin) as in the vector layout."""
    nc = F_site.shape[-1]
    m = np.zeros((4 * nc, 4 * nc), dtype=np.complex128)
    for p, (mu, nu) in enumerate(PLANES):
        m = m + np.kron(F_site[p], sigma_munu(mu, nu))
    return -0.5 * csw * m
