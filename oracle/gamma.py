"""Chiral (Weyl) gamma matrices, entered as printed in App. A (Eq. def_gammamatrices).

Index mu = 0..3 corresponds to the paper's gamma_1..gamma_4.  gamma_5 =
gamma_1 gamma_2 gamma_3 gamma_4 = diag(1,1,-1,-1) (App. A).  The tests check
these entries against the Pauli tensor forms sigma_2 x sigma_1, ..., sigma_1 x
sigma_0 and the Clifford relations, so a mistyped entry is caught.
"""
import numpy as np

_i = 1j

GAMMA = np.array(
    [
        # gamma_1
        [[0, 0, 0, -_i],
         [0, 0, -_i, 0],
         [0, _i, 0, 0],
         [_i, 0, 0, 0]],
        # gamma_2
        [[0, 0, 0, -1],
         [0, 0, 1, 0],
         [0, 1, 0, 0],
         [-1, 0, 0, 0]],
        # gamma_3
        [[0, 0, -_i, 0],
         [0, 0, 0, _i],
         [_i, 0, 0, 0],
         [0, -_i, 0, 0]],
        # gamma_4
        [[0, 0, 1, 0],
         [0, 0, 0, 1],
         [1, 0, 0, 0],
         [0, 1, 0, 0]],
    ],
    dtype=np.complex128,
)

GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]

IDENTITY4 = np.eye(4, dtype=np.complex128)

PAULI = np.array(
    [
        [[1, 0], [0, 1]],
        [[0, 1], [1, 0]],
        [[0, -_i], [_i, 0]],
        [[1, 0], [0, -1]],
    ],
    dtype=np.complex128,
)


def sigma_munu(mu: int, nu: int) -> np.ndarray:
    """sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] (App. A)."""
    g = GAMMA
    return 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])
