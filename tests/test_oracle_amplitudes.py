"""Pins of the oracle's amplitudes: hand-computed circuits, brute force,
the plain definition (state vector), normalisation and order independence."""
import json
import os

import numpy as np
import pytest

import rqcgen
from rqcgen import Circuit, Gate
from oracle import bruteforce as bf
from oracle import peps
from oracle import statevector as sv

S2 = 1 / np.sqrt(2)


def _all_three(c):
    bits = rqcgen.all_bitstrings(c.lv * c.lh)
    a = sv.amplitudes(sv.run(c), bits)
    b = bf.amplitudes(bf.final_vector(c), bits)
    p = peps.amplitudes(peps.build(c), bits)
    return a, b, p


def test_bell_state_by_hand():
    # H q0, H q1, CZ, H q1 on a 1x2 lattice gives (|00> + |11>)/sqrt(2)
    c = Circuit(1, 2, 1, 0, [Gate(0, "H", 0), Gate(0, "H", 1), Gate(1, "CZ", 0, 1), Gate(2, "H", 1)])
    for amps in _all_three(c):
        assert np.allclose(amps, [S2, 0, 0, S2], atol=1e-15)
    # same pair placed vertically (2x1 lattice) and with the gate listed as (1, 0)
    c = Circuit(2, 1, 1, 0, [Gate(0, "H", 0), Gate(0, "H", 1), Gate(1, "CZ", 1, 0), Gate(2, "H", 1)])
    for amps in _all_three(c):
        assert np.allclose(amps, [S2, 0, 0, S2], atol=1e-15)


def test_ghz_by_hand():
    # CNOT = (I x H) CZ (I x H): H q0, then CNOT(0,1), CNOT(1,2) on a 1x3 row
    g = [Gate(0, "H", 0)]
    for a, b in ((0, 1), (1, 2)):
        g += [Gate(1, "H", b), Gate(1, "CZ", a, b), Gate(1, "H", b)]
    c = Circuit(1, 3, 2, 0, g)
    want = np.zeros(8, dtype=complex)
    want[0] = want[7] = S2
    for amps in _all_three(c):
        assert np.allclose(amps, want, atol=1e-15)


def test_qubit_order_by_hand():
    # sqrt(X)^2 = X on qubit 4 of a 2x3 lattice flips exactly that bit
    c = Circuit(2, 3, 1, 0, [Gate(0, "SX", 4), Gate(1, "SX", 4)])
    want = np.zeros(64, dtype=complex)
    want[int("000010", 2)] = 1.0
    for amps in _all_three(c):
        assert np.allclose(amps, want, atol=1e-15)
    # T phase on |1>: H T H on qubit 0 of 1x2
    c = Circuit(1, 2, 1, 0, [Gate(0, "H", 0), Gate(1, "T", 0), Gate(2, "H", 0)])
    w = np.exp(1j * np.pi / 4)
    want = np.array([(1 + w) / 2, 0, (1 - w) / 2, 0])
    for amps in _all_three(c):
        assert np.allclose(amps, want, atol=1e-15)


def test_depth_zero_and_single_layer():
    c = rqcgen.generate(3, 3, 0, 0)   # H layer twice: identity
    for amps in _all_three(c):
        want = np.zeros(512)
        want[0] = 1
        assert np.allclose(amps, want, atol=1e-14)
    c = Circuit(3, 3, 0, 0, [Gate(0, "H", q) for q in range(9)])
    for amps in _all_three(c):
        assert np.allclose(amps, 2 ** -4.5, atol=1e-15)


@pytest.mark.parametrize("lv,lh,d,seed", [(3, 3, 8, 0), (3, 4, 12, 1), (2, 3, 20, 2)])
def test_bruteforce_equals_statevector_equals_peps(lv, lh, d, seed):
    a, b, p = _all_three(rqcgen.generate(lv, lh, d, seed))
    assert np.max(np.abs(a - b)) < 1e-13
    assert np.max(np.abs(a - p)) < 1e-13
    assert abs(np.sum(np.abs(p) ** 2) - 1) < 1e-12


@pytest.mark.parametrize("two_qubit", ["U2", "CZ"])
def test_general_gates(two_qubit):
    c = rqcgen.generate_general(3, 3, 4, 5, two_qubit)
    a, b, p = _all_three(c)
    assert np.max(np.abs(a - b)) < 1e-13
    assert np.max(np.abs(a - p)) < 1e-13
    P = peps.build(c)
    if two_qubit == "U2":
        assert P.chi() > 2


def test_bruteforce_16_qubits():
    c = rqcgen.generate(4, 4, 8, 3)
    bits = rqcgen.bitstrings(4, 4, 3, 32)
    a = sv.amplitudes(sv.run(c), bits)
    b = bf.amplitudes(bf.final_vector(c), bits)
    assert np.max(np.abs(a - b)) < 1e-13


@pytest.mark.parametrize("seed", [0, 1])
def test_peps_rows_vs_statevector_4x5(seed):
    c = rqcgen.generate(4, 5, 24, seed)
    bits = rqcgen.bitstrings(4, 5, seed, 16)
    want = sv.amplitudes(sv.run(c), bits)
    P = peps.build(c)
    assert P.chi() == 8
    for scheme in ("cols", "rows"):
        got = peps.amplitudes(P, bits, scheme)
        assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want)) * 10


def test_contraction_orders_agree_4x4():
    c = rqcgen.generate(4, 4, 16, 4)
    P = peps.build(c)
    bits = rqcgen.bitstrings(4, 4, 4, 6)
    want = sv.amplitudes(sv.run(c), bits)
    for scheme in ("rows", "rows_rl", "rows_bu", "cols", "quadrants"):
        got = peps.amplitudes(P, bits, scheme)
        assert np.max(np.abs(got - want)) < 1e-14, scheme


def test_quadrants_sliced_small():
    c = rqcgen.generate(4, 4, 16, 6)
    P = peps.build(c)
    base = rqcgen.bitstrings(4, 4, 6, 1)[0]
    var = rqcgen.last_row_variants(base, 4, 4, [1, 2, 3])   # col 1 in bl, cols 2-3 in br
    left = var[[0, 4]]            # col 1 = 0 / 1
    right = var[[0, 1, 2, 3]]     # cols 2,3 = 00..11
    res = peps.quadrant_amplitudes_sliced(P, base, left, right)
    want = sv.amplitudes(sv.run(c), var).reshape(2, 4)
    assert np.max(np.abs(res - want)) < 1e-14


def test_quadrants_sliced_6x6_low_depth():
    # two independent contraction orders at the target lattice size
    c = rqcgen.generate(6, 6, 16, 0)
    P = peps.build(c)
    base = rqcgen.bitstrings(6, 6, 0, 1)[0]
    var = rqcgen.last_row_variants(base, 6, 6, [2, 3])
    res = peps.quadrant_amplitudes_sliced(P, base, var[[0, 2]], var[[0, 1]])
    rows = peps.amplitudes(P, var)
    assert np.max(np.abs(res.reshape(-1) - rows)) < 1e-13 * np.max(np.abs(rows))


def test_normalisation_3x3_all_bitstrings():
    c = rqcgen.generate(3, 3, 16, 9)
    P = peps.build(c)
    amps = peps.amplitudes(P, rqcgen.all_bitstrings(9), "rows_bu")
    assert abs(np.sum(np.abs(amps) ** 2) - 1) < 1e-12


def test_chi_bound_eq8():
    for d in (8, 16, 24, 32, 12):
        P = peps.build(rqcgen.generate(4, 4, d, 0))
        dims = peps.bond_dims(P)
        assert P.chi() <= 2 ** -(-d // 8)
        if d % 8 == 0:
            assert P.chi() == 2 ** (d // 8)
            assert set(dims.values()) == {2 ** (d // 8)}


def test_golden_files_match_oracle(golden_dir):
    """Stored goldens were written by tests/golden/make_golden.py (oracle only)."""
    path = os.path.join(golden_dir, "rqc_3x3_d8_s0.json")
    with open(path) as f:
        g = json.load(f)
    c = rqcgen.generate(3, 3, 8, 0)
    assert g["sha256"] == c.sha256()
    bits = np.array(g["bits"], dtype=np.uint8)
    amps = np.array(g["amps_re"]) + 1j * np.array(g["amps_im"])
    assert np.max(np.abs(sv.amplitudes(sv.run(c), bits) - amps)) < 1e-15


@pytest.mark.parametrize("lv,lh,d,seed", [(4, 4, 16, 1), (4, 5, 16, 0), (4, 5, 13, 2), (3, 3, 8, 0), (3, 6, 16, 4)])
def test_row_scheme_with_cut_loops(lv, lh, d, seed):
    """The row scheme with cut loops over v and w (supplement S-II and the
    cut technique) gives the amplitudes of bitstrings that share all rows
    but the last, equal to the state vector (the plain definition)."""
    c = rqcgen.generate(lv, lh, d, seed)
    P = peps.build(c)
    base = rqcgen.bitstrings(lv, lh, seed, 1)[0]
    var = rqcgen.last_row_variants(base, lv, lh, list(range(max(0, lh - 3), lh)))
    got = peps.row_amplitudes_sliced(P, base, var)
    ref = sv.amplitudes(sv.run(c), var)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    bad = var.copy()
    bad[0, 0] ^= 1                                      # differs from the base in row 0
    with pytest.raises(ValueError):
        peps.row_amplitudes_sliced(P, base, bad)


@pytest.mark.parametrize("L,d,seed", [(4, 16, 0), (4, 24, 1), (2, 8, 2)])
def test_square_partition_left_right_halves(L, d, seed):
    """The square partition grouped into left and right halves with cut loops
    over one bond between the upper and one between the lower quadrants (the
    second order of the 6x6 (1+40+1) golden) equals the state vector."""
    c = rqcgen.generate(L, L, d, seed)
    P = peps.build(c)
    bits = rqcgen.bitstrings(L, L, seed, 4)
    got = np.array([peps.halves_amplitude_sliced(P, b) for b in bits])
    ref = sv.amplitudes(sv.run(c), bits)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_6x6_golden_two_orders(golden_dir):
    """The base amplitude of the 6x6 (1+40+1) golden batch from two
    contraction orders of the oracle: the square partition paired top and
    bottom with cut loops over the top e-bond and the last c-bond (eqs.
    S9-S10, rqc_6x6_d40_s0.json) and paired left and right
    (rqc_6x6_d40_s0_halves.json) agree to 1e-12 relative."""
    with open(os.path.join(golden_dir, "rqc_6x6_d40_s0.json")) as f:
        a = json.load(f)
    with open(os.path.join(golden_dir, "rqc_6x6_d40_s0_halves.json")) as f:
        b = json.load(f)
    assert a["sha256"] == b["sha256"] == rqcgen.generate(6, 6, 40, 0).sha256()
    i = a["base_index"]
    assert a["bits"][i] == b["bits"][0] == rqcgen.bitstrings(6, 6, 0, 1)[0].tolist()
    x = complex(a["amps_re"][i], a["amps_im"][i])
    y = complex(b["amps_re"][0], b["amps_im"][0])
    assert abs(x - y) <= 1e-12 * abs(x)
