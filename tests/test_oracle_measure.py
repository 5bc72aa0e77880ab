"""Pins of the oracle's observables and sequential measurement (oracle/measure.py):
closed forms (product states, graph-state stabilizers), an independent
Kronecker-product computation, normalisation, and the sampling statistics
against |psi|^2."""
import numpy as np
import pytest
import scipy.sparse as sp

import rqcgen
from rqcgen import Circuit, Gate
from oracle import bruteforce as bf
from oracle import measure as om
from oracle import statevector as sv

X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
Z = np.diag([1.0, -1.0]).astype(complex)
I2 = np.eye(2, dtype=complex)


def _ry(theta):
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -s], [s, c]], dtype=complex)


def _u1(q, m, cycle=0):
    return Gate(cycle, "U1", q, -1, [float(x) for v in np.asarray(m).reshape(-1) for x in (v.real, v.imag)])


def _product_circuit(thetas):
    return Circuit(1, len(thetas), 1, 0, [_u1(q, _ry(t)) for q, t in enumerate(thetas)], family="product")


def _graph_state(lv, lh):
    gates = [Gate(0, "H", q) for q in range(lv * lh)]
    for r in range(lv):
        for c in range(lh):
            q = r * lh + c
            if c + 1 < lh:
                gates.append(Gate(1, "CZ", q, q + 1))
            if r + 1 < lv:
                gates.append(Gate(1, "CZ", q, q + lh))
    return Circuit(lv, lh, 1, 0, gates, family="graph")


def _neighbours(lv, lh, q):
    r, c = divmod(q, lh)
    out = []
    for dr, dc in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        if 0 <= r + dr < lv and 0 <= c + dc < lh:
            out.append((r + dr) * lh + c + dc)
    return out


def test_product_state_closed_forms():
    th = [0.3, 1.1, 2.0, 2.9]
    psi = sv.run(_product_circuit(th))
    for q, t in enumerate(th):
        assert abs(om.expectation(psi, {q: Z}) - np.cos(t)) < 1e-14
        assert abs(om.expectation(psi, {q: X}) - np.sin(t)) < 1e-14
        assert abs(om.expectation(psi, {q: Y})) < 1e-14
        assert abs(om.marginal(psi, [q], [0]) - np.cos(t / 2) ** 2) < 1e-14
    assert abs(om.expectation(psi, {0: Z, 2: X}) - np.cos(th[0]) * np.sin(th[2])) < 1e-14
    assert abs(om.expectation(psi, {}) - 1) < 1e-14


def test_graph_state_stabilizers():
    """H on every qubit then CZ on every lattice edge: the stabilizers
    X_a prod_{b ~ a} Z_b have expectation 1; a single X_a or a Z_a Z_b on an
    edge has expectation 0; Y_a prod_{b ~ a} Z_b (= i X_a Z_a ...) has 0."""
    lv, lh = 2, 3
    psi = sv.run(_graph_state(lv, lh))
    for a in range(lv * lh):
        ops = {a: X}
        for b in _neighbours(lv, lh, a):
            ops[b] = Z
        assert abs(om.expectation(psi, ops) - 1) < 1e-13
        assert abs(om.expectation(psi, {a: X})) < 1e-13
        ops[a] = Y
        assert abs(om.expectation(psi, ops)) < 1e-13
    assert abs(om.expectation(psi, {0: Z, 1: Z})) < 1e-13


def _kron_expectation(c, ops):
    """The same value by explicit Kronecker products on the brute-force
    vector (qubit 0 the most significant factor)."""
    n = c.lv * c.lh
    v = bf.final_vector(c)
    f = [sp.csr_matrix(ops.get(q, I2)) for q in range(n)]
    O = f[0]
    for m in f[1:]:
        O = sp.kron(O, m, format="csr")
    return complex(np.vdot(v, O @ v))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_expectation_vs_kronecker_products(seed):
    rng = np.random.default_rng(seed)
    c = rqcgen.generate_general(2, 3, 3, seed, "U2")
    psi = sv.run(c)
    for _ in range(4):
        qs = rng.choice(6, size=3, replace=False)
        ops = {int(q): rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)) for q in qs}
        assert abs(om.expectation(psi, ops) - _kron_expectation(c, ops)) < 1e-13
        # <O^dagger> = conj <O>
        dag = {q: m.conj().T for q, m in ops.items()}
        assert abs(om.expectation(psi, dag) - np.conj(om.expectation(psi, ops))) < 1e-13


def test_marginals_normalise_and_reduce_to_amplitudes():
    c = rqcgen.generate(3, 3, 8, 4)
    psi = sv.run(c)
    tot = sum(om.marginal(psi, [1, 4, 8], [a, b, d]) for a in (0, 1) for b in (0, 1) for d in (0, 1))
    assert abs(tot - 1) < 1e-13
    bits = rqcgen.bitstrings(3, 3, 4, 5)
    amps = sv.amplitudes(psi, bits)
    for b, a in zip(bits, amps):
        assert abs(om.marginal(psi, range(9), b) - abs(a) ** 2) < 1e-15
    # <Z_q> = p(q = 0) - p(q = 1)
    for q in range(9):
        assert abs(om.expectation(psi, {q: Z}) - (om.marginal(psi, [q], [0]) - om.marginal(psi, [q], [1]))) < 1e-13


def test_sampling_product_state_is_independent_thresholds():
    th = np.array([0.4, 1.3, 2.2, 2.8, 1.9])
    psi = sv.run(_product_circuit(th))
    u = np.random.default_rng(3).random((50, 5))
    bits, prob = om.sample_sequential(psi, u)
    p0 = np.cos(th / 2) ** 2
    assert np.array_equal(bits, (u >= p0[None, :]).astype(np.uint8))
    want = np.prod(np.where(bits == 0, p0[None, :], 1 - p0[None, :]), axis=1)
    assert np.allclose(prob, want, rtol=1e-13, atol=0)


def test_sampling_basis_state_is_deterministic():
    c = Circuit(2, 2, 1, 0, [_u1(0, X), _u1(3, X)], family="basis")
    u = np.random.default_rng(4).random((20, 4))
    bits, prob = om.sample_sequential(sv.run(c), u)
    assert (bits == np.array([1, 0, 0, 1], dtype=np.uint8)).all()
    assert np.allclose(prob, 1.0)


def test_sampling_frequencies_follow_born_rule():
    """Many draws on a 3-qubit state: the frequencies of the 8 outcomes
    against |psi|^2 (chi-square, fixed seed), and p(bits) == |psi(bits)|^2."""
    c = rqcgen.generate_general(1, 3, 3, 9, "U2")
    psi = sv.run(c)
    u = np.random.default_rng(5).random((40000, 3))
    bits, prob = om.sample_sequential(psi, u)
    p = (np.abs(psi) ** 2).reshape(-1)
    idx = bits[:, 0] * 4 + bits[:, 1] * 2 + bits[:, 2]
    assert np.allclose(prob, p[idx], rtol=1e-12, atol=0)
    counts = np.bincount(idx, minlength=8)
    exp = p * len(u)
    chi2 = float(np.sum((counts - exp) ** 2 / exp))
    assert chi2 < 24.3  # 7 degrees of freedom, p = 0.001


def test_projection_norm_is_the_marginal_and_idempotent():
    c = rqcgen.generate(3, 3, 8, 6)
    psi = sv.run(c)
    for q in (0, 4, 8):
        for v in (0, 1):
            ph = om.project(psi, q, v)
            assert abs(np.vdot(ph, ph).real - om.marginal(psi, [q], [v])) < 1e-14
            assert np.array_equal(om.project(ph, q, v), ph)
            assert not np.any(np.take(ph, 1 - v, axis=q))
    # the two outcomes add back to the state
    assert np.allclose(om.project(psi, 2, 0) + om.project(psi, 2, 1), psi, atol=0)
