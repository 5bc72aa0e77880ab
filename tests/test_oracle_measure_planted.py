"""Plant plausible mistakes in the oracle's observables and sequential
measurement (on the CPU) and check that the pins of test_oracle_measure.py
catch each one: the pinned test, run against the planted variant, must fail."""
import numpy as np
import pytest

import test_oracle_measure as pins
from oracle import measure as om
from oracle.statevector import apply_1q


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_pins_pass_on_the_oracle():
    pins.test_product_state_closed_forms()
    pins.test_expectation_vs_kronecker_products(0)
    pins.test_marginals_normalise_and_reduce_to_amplitudes()
    pins.test_sampling_product_state_is_independent_thresholds()
    pins.test_sampling_frequencies_follow_born_rule()
    pins.test_projection_norm_is_the_marginal_and_idempotent()


def test_bra_without_conjugate_is_caught(monkeypatch):
    def bad(psi, ops):
        phi = psi
        for q, o in ops.items():
            phi = apply_1q(phi, np.asarray(o, dtype=np.complex128), q)
        return complex(np.dot(psi.reshape(-1), phi.reshape(-1)))
    monkeypatch.setattr(om, "expectation", bad)
    _fails(pins.test_expectation_vs_kronecker_products, 0)


def test_transposed_operator_is_caught(monkeypatch):
    def bad(psi, ops):
        phi = psi
        for q, o in ops.items():
            phi = apply_1q(phi, np.asarray(o, dtype=np.complex128).T, q)
        return complex(np.vdot(psi.reshape(-1), phi.reshape(-1)))
    monkeypatch.setattr(om, "expectation", bad)
    _fails(pins.test_expectation_vs_kronecker_products, 1)


def test_reversed_qubit_order_is_caught(monkeypatch):
    def bad(psi, ops):
        phi = psi
        for q, o in ops.items():
            phi = apply_1q(phi, np.asarray(o, dtype=np.complex128), psi.ndim - 1 - q)
        return complex(np.vdot(psi.reshape(-1), phi.reshape(-1)))
    monkeypatch.setattr(om, "expectation", bad)
    _fails(pins.test_product_state_closed_forms)


def test_marginal_of_moduli_is_caught(monkeypatch):
    def bad(psi, qubits, values):
        p = np.abs(psi)
        idx = [slice(None)] * psi.ndim
        for q, v in zip(qubits, values):
            idx[q] = int(v)
        return float(np.sum(p[tuple(idx)]))
    monkeypatch.setattr(om, "marginal", bad)
    _fails(pins.test_marginals_normalise_and_reduce_to_amplitudes)


def test_projection_on_the_other_outcome_is_caught(monkeypatch):
    def bad(psi, qubit, value):
        out = np.array(psi, copy=True)
        idx = [slice(None)] * psi.ndim
        idx[qubit] = int(value)
        out[tuple(idx)] = 0
        return out
    monkeypatch.setattr(om, "project", bad)
    _fails(pins.test_projection_norm_is_the_marginal_and_idempotent)


def test_flipped_threshold_is_caught(monkeypatch):
    """Outcome 0 taken when u lies above p0 / (p0 + p1) instead of below."""
    def bad(psi, u):
        u = np.asarray(u, dtype=np.float64)
        S, N = u.shape
        bits = np.zeros((S, N), dtype=np.uint8)
        probs = np.zeros(S)
        for s in range(S):
            cond = np.abs(psi) ** 2
            for k in range(N):
                p0, p1 = float(np.sum(cond[0])), float(np.sum(cond[1]))
                b = 0 if u[s, k] >= p0 / (p0 + p1) else 1
                bits[s, k] = b
                cond = cond[b]
                probs[s] = p1 if b else p0
        return bits, probs
    monkeypatch.setattr(om, "sample_sequential", bad)
    _fails(pins.test_sampling_product_state_is_independent_thresholds)


def test_unconditioned_thresholds_are_caught(monkeypatch):
    """Each qubit drawn from its own one-qubit marginal, ignoring the earlier
    outcomes: right for product states, wrong for entangled ones."""
    def bad(psi, u):
        u = np.asarray(u, dtype=np.float64)
        S, N = u.shape
        p_all = np.abs(psi) ** 2
        bits = np.zeros((S, N), dtype=np.uint8)
        probs = np.ones(S)
        for k in range(N):
            p0 = float(np.sum(np.take(p_all, 0, axis=k)))
            p1 = float(np.sum(np.take(p_all, 1, axis=k)))
            b = (u[:, k] >= p0 / (p0 + p1)).astype(np.uint8)
            bits[:, k] = b
            probs *= np.where(b == 1, p1, p0)
        return bits, probs
    monkeypatch.setattr(om, "sample_sequential", bad)
    pins.test_sampling_product_state_is_independent_thresholds()   # not caught there ...
    _fails(pins.test_sampling_frequencies_follow_born_rule)         # ... but here
