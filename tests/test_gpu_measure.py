"""GPU parity of observables and sequential measurement through the
double-layer network (psim_double_layer, psim_sample): expectation values,
marginals and sampled bitstrings against the oracle's plain definitions on the
state vector, in every precision and with the row scheme and the square
partition."""
import sys

import numpy as np
import pytest

import rqcgen
from oracle import measure as om
from oracle import statevector as sv

pytestmark = pytest.mark.gpu

X = np.array([[0, 1], [1, 0]], dtype=complex)
Z = np.diag([1.0, -1.0]).astype(complex)
BAR = {"fp64": 1e-11, "fp32": 2e-5, "fp32_3m": 2e-5, "fp32_3ms": 2e-5}
# fp32_3ms: FP32 3M with split accumulation
KW = {"fp64": {"prec": "fp64"}, "fp32": {"prec": "fp32"}, "fp32_3m": {"prec": "fp32_3m"},
      "fp32_3ms": {"prec": "fp32_3m", "split_acc": True}}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ps():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1905_08394_amd as ps
    ps.lib()
    return ps


CIRCUITS = [("rqc", 3, 3, 8, 0), ("rqc", 3, 4, 13, 1), ("rqc", 4, 4, 12, 2), ("U2", 2, 5, 2, 3)]


def _circuit(kind, lv, lh, d, seed):
    return rqcgen.generate(lv, lh, d, seed) if kind == "rqc" else rqcgen.generate_general(lv, lh, d, seed, "U2")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_3m", "fp32_3ms"])
@pytest.mark.parametrize("sweep", [0, 3])
@pytest.mark.parametrize("case", CIRCUITS)
def test_expectation_values(ps, case, sweep, prec):
    """<psi|psi> = 1, <Z_q>, <X_q>, a two-site product and a random complex
    operator on three sites, each one contraction of the double-layer
    network, against the state vector."""
    c = _circuit(*case)
    n = c.lv * c.lh
    psi = sv.run(c)
    rng = np.random.default_rng(case[4])
    P = ps.Peps(c)
    kw = dict(KW[prec], sweep=sweep)
    qs = rng.choice(n, size=3, replace=False)
    rand = {int(q): rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)) for q in qs}
    cases = [{}, {0: Z}, {n - 1: X}, {1: Z, n - 2: X}, rand]
    worst = 0.0
    for ops in cases:
        got = ps.expectation(P, ops, **kw)
        want = om.expectation(psi, ops)
        worst = max(worst, abs(got - want))
        assert abs(got - want) <= BAR[prec] * max(1.0, abs(want)), (ops.keys(), got, want)
    say(f"expectation {case} sweep {sweep} {prec}: max |error| {worst:.2e}")


@pytest.mark.parametrize("prec", ["fp64", "fp32_3m"])
def test_marginals_as_amplitudes_of_the_double_layer(ps, prec):
    """One double-layer PEPS with slices (|0><0|, |1><1|) on four sites and
    (I, I) elsewhere: its amplitudes over all 16 values of those sites are
    the marginals p(t_S), batched through one plan."""
    c = rqcgen.generate(3, 4, 13, 5)
    n = 12
    psi = sv.run(c)
    S = [0, 5, 6, 11]
    o = np.zeros((n, 2, 2, 2), dtype=complex)
    o[:, :] = np.eye(2)
    for q in S:
        o[q, 0] = np.diag([1.0, 0.0])
        o[q, 1] = np.diag([0.0, 1.0])
    P = ps.Peps(c)
    V = P.double_layer(o)
    info = V.info()
    assert info["bond_dims"] == [b * b for b in P.info()["bond_dims"]]
    vals = rqcgen.all_bitstrings(4)
    bits = np.zeros((16, n), dtype=np.uint8)
    bits[:, S] = vals
    got = ps.Plan(V, prec=prec, max_batch=16).amplitudes(bits)
    want = np.array([om.marginal(psi, S, v) for v in vals])
    assert np.max(np.abs(got.imag)) <= BAR[prec]
    assert np.max(np.abs(got.real - want)) <= BAR[prec], np.max(np.abs(got.real - want))
    assert abs(got.real.sum() - 1) <= 4 * BAR[prec]


@pytest.mark.parametrize("prec,sweep", [("fp64", 0), ("fp64", 3), ("fp32_3m", 0)])
@pytest.mark.parametrize("lv,lh,d,seed", [(3, 3, 8, 0), (3, 4, 13, 1), (4, 4, 12, 2)])
def test_sequential_measurement(ps, lv, lh, d, seed, prec, sweep):
    """psim_sample with the same uniforms as the oracle's sequential
    measurement: every decision agrees except where u lies within the
    precision's bar of the threshold (checked: then both outcomes are valid);
    p(bits) agrees with |psi(bits)|^2."""
    c = rqcgen.generate(lv, lh, d, seed)
    n = lv * lh
    psi = sv.run(c)
    u = np.random.default_rng(100 + seed).random((64, n))
    bits, prob = ps.sample(ps.Peps(c), u, prec=prec, sweep=sweep, max_batch=128)
    obits, oprob = om.sample_sequential(psi, u)
    p_all = np.abs(psi) ** 2
    tol = 1e-9 if prec == "fp64" else 1e-3
    atol, rtol = (1e-13, 1e-9) if prec == "fp64" else (1e-6, 1e-3)
    mism = 0
    for s in range(len(u)):
        if np.array_equal(bits[s], obits[s]):
            continue
        # first differing qubit: u must sit on the oracle's threshold there
        k = int(np.nonzero(bits[s] != obits[s])[0][0])
        cond = p_all[tuple(int(b) for b in obits[s][:k])]
        t = float(np.sum(cond[0])) / float(np.sum(cond))
        assert abs(u[s, k] - t) <= tol, (s, k, u[s, k], t)
        mism += 1
    ok = np.all(bits == obits, axis=1)
    assert np.allclose(prob[ok], oprob[ok], rtol=rtol, atol=atol)
    assert np.allclose(prob, p_all[tuple(bits.T)], rtol=rtol, atol=atol)
    say(f"sample {lv}x{lh} d{d} {prec} sweep {sweep}: {len(u) - mism}/{len(u)} identical to the oracle")
    assert mism <= 2


def test_sample_zero_samples_and_repeat(ps):
    """No samples: nothing written; the same uniforms twice: the same bits."""
    c = rqcgen.generate(3, 3, 8, 4)
    P = ps.Peps(c)
    bits, prob = ps.sample(P, np.zeros((0, 9)), prec="fp64")
    assert bits.shape == (0, 9) and prob.shape == (0,)
    u = np.random.default_rng(8).random((16, 9))
    b1, p1 = ps.sample(P, u, prec="fp64", max_batch=32)
    b2, p2 = ps.sample(P, u, prec="fp64", max_batch=32)
    assert np.array_equal(b1, b2) and np.array_equal(p1, p2)


def _sv_apply(psi, gates):
    from oracle import gates as G
    for g in gates:
        m = G.matrix_of(g)
        psi = sv.apply_2q(psi, m, g.q0, g.q1) if G.is_two_qubit(g) else sv.apply_1q(psi, m, g.q0)
    return psi


@pytest.mark.parametrize("prec,sweep", [("fp64", 0), ("fp64", 3), ("fp32_3m", 0)])
def test_measurements_with_gates_in_between(ps, prec, sweep):
    """Measure a qubit (double-layer probability, outcome from a fixed
    uniform), record it on the PEPS, apply more gates, measure another: every
    probability and the final unnormalised amplitudes against the oracle doing
    the same on the state vector (the remark after eq. 7)."""
    c = rqcgen.generate(3, 4, 8, 2)
    more = rqcgen.generate_general(3, 4, 2, 5, "U2").gates
    n = 12
    P = ps.Peps(c)
    psi = sv.run(c)
    P0 = np.diag([1.0, 0.0]).astype(complex)
    tol = 1e-11 if prec == "fp64" else 2e-5
    kw = dict(prec=prec, sweep=sweep)
    for q, u, gates in ((5, 0.37, more), (2, 0.61, ())):
        norm = ps.expectation(P, {}, **kw).real
        p0 = ps.expectation(P, {q: P0}, **kw).real / norm
        o_norm = np.vdot(psi, psi).real
        o_p0 = om.marginal(psi, [q], [0]) / o_norm
        assert abs(p0 - o_p0) <= tol, (q, p0, o_p0)
        assert abs(norm - o_norm) <= tol * max(1.0, o_norm)
        t = 0 if u < o_p0 else 1
        P.project(q, t)
        psi = om.project(psi, q, t)
        if gates:
            P.apply(gates)
            psi = _sv_apply(psi, gates)
    bits = rqcgen.bitstrings(3, 4, 2, 24)
    a = ps.Plan(P, prec=prec, sweep=sweep, max_batch=len(bits)).amplitudes(bits)
    ref = sv.amplitudes(psi, bits)
    scale = np.sqrt(np.vdot(psi, psi).real)
    assert np.max(np.abs(a - ref)) * 2 ** (n / 2) <= tol * 10 * scale, np.max(np.abs(a - ref))
