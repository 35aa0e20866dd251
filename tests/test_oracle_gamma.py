"""Pins for the chiral gamma matrices (App. A) against independent printed data."""
import os

import numpy as np
import pytest

from oracle.gamma import GAMMA, GAMMA5, IDENTITY4, PAULI, sigma_munu

pytestmark = pytest.mark.filterwarnings("ignore")


def _entry(tok):
    return {"1": 1, "-1": -1, "i": 1j, "-i": -1j, "0": 0}[tok]


def test_tensor_forms():
    # gamma_1..4 = s2(x)s1, s2(x)s2, s2(x)s3, s1(x)s0 with the first factor on the 2x2 block index
    forms = [(2, 1), (2, 2), (2, 3), (1, 0)]
    for mu, (a, b) in enumerate(forms):
        np.testing.assert_array_equal(GAMMA[mu], np.kron(PAULI[a], PAULI[b]))


def test_clifford_and_gamma5():
    for mu in range(4):
        assert np.allclose(GAMMA[mu], GAMMA[mu].conj().T)
        for nu in range(4):
            anti = GAMMA[mu] @ GAMMA[nu] + GAMMA[nu] @ GAMMA[mu]
            assert np.allclose(anti, 2.0 * (mu == nu) * IDENTITY4)
    np.testing.assert_allclose(GAMMA5, np.diag([1, 1, -1, -1]), atol=1e-15)


def test_projectors_printed(golden_dir):
    with open(os.path.join(golden_dir, "appA_projectors.txt")) as f:
        lines = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    seen = 0
    for toks in lines:
        mu, which = int(toks[0]) - 1, toks[1]
        rows = " ".join(toks[2:]).split("|")
        m = np.array([[_entry(t) for t in r.split()] for r in rows], dtype=complex) / np.sqrt(2)
        sign = +1 if which == "P" else -1
        np.testing.assert_allclose(m @ m.conj().T, 0.5 * (IDENTITY4 + sign * GAMMA[mu]), atol=1e-15)
        np.testing.assert_allclose(m.conj().T @ m, np.eye(2), atol=1e-15)
        seen += 1
    assert seen == 8


def test_sigma_printed(golden_dir):
    with open(os.path.join(golden_dir, "appA_sigma.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 6
    for mu, nu, sign, a, b in rows:
        expect = float(sign) * np.kron(PAULI[int(a)], PAULI[int(b)])
        np.testing.assert_allclose(sigma_munu(int(mu) - 1, int(nu) - 1), expect, atol=1e-15)
