"""O1: brute force with explicit 2^N x 2^N operators (N <= 16).

Each gate becomes a sparse operator on the whole register built from
Kronecker products, with qubit 0 the most significant factor.  A two-qubit
matrix O is expanded in elementary matrices,
    O = sum_{a,b,c,d} O[2a+b, 2c+d] |a><c|_{q0} (x) |b><d|_{q1},
so that any qubit pair (adjacent or not, in either order) uses the same code.
This index logic is deliberately different from the state-vector module.
"""
import numpy as np
import scipy.sparse as sp

from . import gates as G


def _elem(a: int, c: int) -> sp.csr_matrix:
    m = np.zeros((2, 2), dtype=np.complex128)
    m[a, c] = 1.0
    return sp.csr_matrix(m)


def _kron_all(factors):
    out = factors[0]
    for f in factors[1:]:
        out = sp.kron(out, f, format="csr")
    return out


def operator(gate, n: int) -> sp.csr_matrix:
    eye = sp.identity(2, dtype=np.complex128, format="csr")
    m = G.matrix_of(gate)
    if not G.is_two_qubit(gate):
        f = [eye] * n
        f[gate.q0] = sp.csr_matrix(m)
        return _kron_all(f)
    total = None
    for a in range(2):
        for b in range(2):
            for c in range(2):
                for d in range(2):
                    coef = m[2 * a + b, 2 * c + d]
                    if coef == 0:
                        continue
                    f = [eye] * n
                    f[gate.q0] = _elem(a, c)
                    f[gate.q1] = _elem(b, d)
                    term = coef * _kron_all(f)
                    total = term if total is None else total + term
    return total


def final_vector(circuit) -> np.ndarray:
    """Final state as a flat vector, index = sum_n tau_n 2^(N-1-n)."""
    n = circuit.lv * circuit.lh
    if n > 16:
        raise ValueError("brute force is limited to 16 qubits")
    v = np.zeros(2 ** n, dtype=np.complex128)
    v[0] = 1.0
    for g in circuit.gates:
        v = operator(g, n) @ v
    return v


def amplitudes(vec: np.ndarray, bits: np.ndarray) -> np.ndarray:
    bits = np.asarray(bits, dtype=np.int64)
    n = bits.shape[1]
    weights = 2 ** np.arange(n - 1, -1, -1, dtype=np.int64)
    return vec[bits @ weights]
