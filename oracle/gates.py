"""Gate matrices of the random circuits, written out from their definitions.

The circuits use the Hadamard H, T = diag(1, e^{i pi/4}), the square roots
X^{1/2} and Y^{1/2}, and the controlled-Z (supplement S-I).  The paper names
the gates without matrices; we take the principal square roots, for which
sqrt(X)^2 = X and sqrt(Y)^2 = Y hold exactly.  Two-qubit matrices act on
(q0, q1) with row index 2*tau_q0 + tau_q1.
"""
import numpy as np

SQ2 = np.sqrt(2.0)

H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / SQ2
T = np.array([[1, 0], [0, np.exp(1j * np.pi / 4)]], dtype=np.complex128)
SX = 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128)
SY = 0.5 * np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]], dtype=np.complex128)
CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)

NAMED = {"H": H, "T": T, "SX": SX, "SY": SY, "CZ": CZ}


def matrix_of(gate) -> np.ndarray:
    """Matrix of an rqcgen.Gate: named gates or the explicit U1/U2 payload."""
    if gate.kind in NAMED:
        return NAMED[gate.kind]
    if gate.kind in ("U1", "U2"):
        dim = 2 if gate.kind == "U1" else 4
        v = np.asarray(gate.m, dtype=np.float64)
        if v.size != 2 * dim * dim:
            raise ValueError("gate matrix has the wrong size")
        return (v[0::2] + 1j * v[1::2]).reshape(dim, dim)
    raise ValueError(f"unknown gate kind {gate.kind}")


def is_two_qubit(gate) -> bool:
    return gate.kind in ("CZ", "U2")
