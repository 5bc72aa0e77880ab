"""O2: state-vector simulation, the plain definition of an amplitude.

amplitude(tau) = <tau| G_K ... G_1 |0...0>, the quantity the PEPS overlap of
eq. (7) / (S1) computes exactly.  The state is an array of shape (2,)*N whose
axis n is qubit n; gates are applied with tensordot in circuit order.
Practical up to about 28 qubits in FP64.
"""
import numpy as np

from . import gates as G


def initial_state(n: int) -> np.ndarray:
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    return psi


def apply_1q(psi: np.ndarray, u: np.ndarray, q: int) -> np.ndarray:
    out = np.tensordot(u, psi, axes=([1], [q]))  # new axis 0 = tau_q
    return np.moveaxis(out, 0, q)


def apply_2q(psi: np.ndarray, o: np.ndarray, q0: int, q1: int) -> np.ndarray:
    o4 = o.reshape(2, 2, 2, 2)  # [tau0, tau1, sigma0, sigma1]
    out = np.tensordot(o4, psi, axes=([2, 3], [q0, q1]))
    return np.moveaxis(out, [0, 1], [q0, q1])


def run(circuit) -> np.ndarray:
    """Final state as an array of shape (2,)*N."""
    n = circuit.lv * circuit.lh
    psi = initial_state(n)
    for g in circuit.gates:
        m = G.matrix_of(g)
        if G.is_two_qubit(g):
            psi = apply_2q(psi, m, g.q0, g.q1)
        else:
            psi = apply_1q(psi, m, g.q0)
    return psi


def amplitudes(psi: np.ndarray, bits: np.ndarray) -> np.ndarray:
    """Amplitudes <tau|psi> for each row tau of bits (shape (B, N))."""
    bits = np.asarray(bits)
    return np.array([psi[tuple(int(b) for b in row)] for row in bits], dtype=np.complex128)
