"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins
catch them: each planted variant must disagree with the plain definition."""
import numpy as np

import rqcgen
from oracle import gates as G
from oracle import peps
from oracle import statevector as sv


def _peps_error(circuit, bits):
    want = sv.amplitudes(sv.run(circuit), bits)
    got = peps.amplitudes(peps.build(circuit), bits)
    return np.max(np.abs(got - want))


CIRC = rqcgen.generate(3, 3, 16, 2)
BITS = rqcgen.all_bitstrings(9)[::7]


def test_reference_is_clean():
    assert _peps_error(CIRC, BITS) < 1e-13


def test_mismatched_bundling_is_caught(monkeypatch):
    orig = peps.apply_2q

    def bad(p, o, q0, q1):
        orig(p, o, q0, q1)
        # reinterpret the right/lower site's bundled leg as (new, old)
        (r0, c0), (r1, c1) = p.pos(q0), p.pos(q1)
        m = max(q0, q1)
        a = p.A[m]
        if r0 == r1:
            _, l, r, u, d = a.shape
            if l % 2 == 0 and l > 2:
                p.A[m] = a.reshape(2, l // 2, 2, r, u, d).transpose(0, 2, 1, 3, 4, 5).reshape(a.shape)
    monkeypatch.setattr(peps, "apply_2q", bad)
    assert _peps_error(CIRC, BITS) > 1e-3


def test_rank_one_split_is_caught(monkeypatch):
    orig = peps.svd_split

    def bad(o, tol=1e-12):
        un, vm = orig(o, tol)
        return un[:, :, :1], vm[:1]
    monkeypatch.setattr(peps, "svd_split", bad)
    assert _peps_error(CIRC, BITS) > 1e-3


def test_transposed_factor_is_caught(monkeypatch):
    orig = peps.svd_split

    def bad(o, tol=1e-12):
        un, vm = orig(o, tol)
        return un.transpose(1, 0, 2), vm
    monkeypatch.setattr(peps, "svd_split", bad)
    c = rqcgen.generate_general(2, 3, 3, 1)
    assert _peps_error(c, rqcgen.all_bitstrings(6)) > 1e-3


def test_wrong_sign_in_gate_is_caught():
    bad_sy = 0.5 * np.array([[1 + 1j, 1 + 1j], [1 + 1j, 1 + 1j]])
    y = np.array([[0, -1j], [1j, 0]])
    assert not np.allclose(bad_sy @ bad_sy, y)
    assert np.allclose(G.SY @ G.SY, y)


def test_dropped_site_is_caught(monkeypatch):
    orig = peps.site_order

    def bad(lv, lh, scheme):
        return orig(lv, lh, scheme)[:-1]
    monkeypatch.setattr(peps, "site_order", bad)
    try:
        err = _peps_error(CIRC, BITS)
    except AssertionError:
        return  # the contraction no longer reduces to a scalar
    assert err > 1e-3


def test_sliced_quadrants_dropped_slice_is_caught(monkeypatch):
    """One slice of the cut loop over the top bond lost from T (the
    square-partition oracle that wrote the 6x6 golden values)."""
    import pytest
    import test_oracle_amplitudes as pins
    orig = peps._accumulate_matmul
    calls = []

    def bad(c, a, b, rows=4096):
        calls.append(1)
        if len(calls) != 2:
            orig(c, a, b, rows)
    monkeypatch.setattr(peps, "_accumulate_matmul", bad)
    with pytest.raises(AssertionError):
        pins.test_quadrants_sliced_small()
    assert len(calls) > 2


def test_sliced_quadrants_shifted_bottom_slice_is_caught(monkeypatch):
    """The lower-left quadrant sliced at z + 1 where the lower-right one is
    sliced at z (an off-by-one between the two sides of the cut loop)."""
    import pytest
    import test_oracle_amplitudes as pins
    orig = peps.contract_sites

    def bad(sites, order, start=None, fixed=None):
        order = list(order)
        if fixed and order and order[0] == (3, 0):          # lower-left quadrant of 4x4
            (lab, z), = fixed.items()
            fixed = {lab: (z + 1) % 4}
        return orig(sites, order, start, fixed)
    monkeypatch.setattr(peps, "contract_sites", bad)
    with pytest.raises(AssertionError):
        pins.test_quadrants_sliced_small()
