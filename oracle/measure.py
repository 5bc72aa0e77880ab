"""Observables and sequential measurement of a state vector: the plain
definitions the double-layer contractions must reproduce (test
infrastructure only, like the rest of oracle/).

The main text (the remark after eq. 7, and the conclusions) notes that the
simulator keeps the whole state, so it yields expectation values and
sequences of measurements besides single amplitudes: measure one qubit
(probabilities of |0> and |1>), project a copy of the state on the outcome,
measure the next qubit, and so on.  Written out on the state vector psi
(shape (2,)*N, axis n = qubit n):
  <psi| prod_n O_n |psi>                 one-qubit operators on any sites;
  p(t_S) = sum over the other qubits of |psi|^2 with qubits S fixed to t_S;
  sequential measurement, qubit 0 first: qubit k is 0 when the caller's
  uniform number u_k is below p(t_0..t_{k-1}, 0) / p(t_0..t_{k-1}) (taking
  the denominator as p(.., 0) + p(.., 1)).
"""
import numpy as np

from .statevector import apply_1q


def expectation(psi: np.ndarray, ops: dict) -> complex:
    """<psi| prod_n ops[n] |psi> for a dict {qubit: 2x2 matrix} (conclusions:
    expectation values of the stored state)."""
    phi = psi
    for q, o in ops.items():
        phi = apply_1q(phi, np.asarray(o, dtype=np.complex128), q)
    return complex(np.vdot(psi.reshape(-1), phi.reshape(-1)))


def marginal(psi: np.ndarray, qubits, values) -> float:
    """Probability that measuring the given qubits yields the given values
    (the probabilities the remark after eq. 7 computes qubit by qubit)."""
    p = np.abs(psi) ** 2
    idx = [slice(None)] * psi.ndim
    for q, v in zip(qubits, values):
        idx[q] = int(v)
    return float(np.sum(p[tuple(idx)]))


def project(psi: np.ndarray, qubit: int, value: int) -> np.ndarray:
    """The state after measuring qubit with outcome value, unnormalised
    (the copy projected on the outcome in the remark after eq. 7): entries
    whose qubit differs from value set to zero."""
    out = np.array(psi, copy=True)
    idx = [slice(None)] * psi.ndim
    idx[qubit] = 1 - int(value)
    out[tuple(idx)] = 0
    return out


def sample_sequential(psi: np.ndarray, u: np.ndarray):
    """Bitstrings drawn qubit by qubit with the given uniforms u (shape
    (S, N)), the measured qubit projected before the next is measured (the
    remark after eq. 7); returns (bits (S, N) uint8, p(bits) per sample)."""
    u = np.asarray(u, dtype=np.float64)
    S, N = u.shape
    p_all = np.abs(psi) ** 2
    bits = np.zeros((S, N), dtype=np.uint8)
    probs = np.zeros(S)
    for s in range(S):
        cond = p_all  # distribution restricted to the prefix drawn so far
        p_pref = 1.0
        for k in range(N):
            # axis 0 of cond is qubit k once the earlier axes are fixed
            p0 = float(np.sum(cond[0]))
            p1 = float(np.sum(cond[1]))
            t = p0 / (p0 + p1) if p0 + p1 > 0 else 0.5
            b = 0 if u[s, k] < t else 1
            bits[s, k] = b
            cond = cond[b]
            p_pref = p1 if b else p0
        probs[s] = p_pref
    return bits, probs
