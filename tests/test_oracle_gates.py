"""Pins of the oracle's gate matrices against textbook algebra."""
import numpy as np

from oracle import gates as G
from oracle import peps

# Pauli matrices typed independently of the oracle
X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
Z = np.array([[1, 0], [0, -1]], dtype=complex)
I2 = np.eye(2)


def test_unitary():
    for m in (G.H, G.T, G.SX, G.SY, G.CZ):
        assert np.allclose(m.conj().T @ m, np.eye(m.shape[0]), atol=1e-15)


def test_square_roots_and_identities():
    assert np.array_equal(G.SX @ G.SX, X)
    assert np.array_equal(G.SY @ G.SY, Y)
    assert np.allclose(G.T @ G.T, np.diag([1, 1j]), atol=1e-15)
    assert np.allclose(G.H @ G.H, I2, atol=1e-15)
    assert np.allclose(G.H @ X @ G.H, Z, atol=1e-15)
    # CZ = |0><0| (x) I + |1><1| (x) Z
    p0, p1 = np.diag([1, 0]), np.diag([0, 1])
    assert np.array_equal(G.CZ, np.kron(p0, I2) + np.kron(p1, Z))


def test_svd_split_reconstructs():
    rng = np.random.default_rng(0)
    cases = [G.CZ]
    for _ in range(5):
        z = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
        q, _ = np.linalg.qr(z)
        cases.append(q)
    for o in cases:
        un, vm = peps.svd_split(o)
        # un[tn, sn, s], vm[s, tm, sm] -> O[tn, tm, sn, sm] -> O[(tn tm), (sn sm)]
        o4 = np.einsum("ask,kbt->abst", un, vm).reshape(4, 4)
        assert np.allclose(o4, o, atol=1e-14)
    un, vm = peps.svd_split(G.CZ)
    assert un.shape[2] == 2, "a controlled gate has operator-Schmidt rank 2 (eq. 4)"
