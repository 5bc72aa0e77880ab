"""GPU parity of the square partition (supplement S-II, Fig. S2(b), eqs.
S9-S10): four quadrant contractions joined by two D^h x D^h x D^h complex
GEMMs and a final inner product, against the oracle (state vector up to 16
qubits, the oracle's PEPS contraction above, the 6x6 (1+40+1) golden values
from the oracle's sliced square partition) and against the row scheme."""
import json
import os
import sys

import numpy as np
import pytest

import rqcgen
from oracle import peps as opeps
from oracle import statevector as sv

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
AMP_BAR = {"fp64": 1e-10, "fp32": 1e-5, "fp32_3m": 1e-5}


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


def _eps_rms(a, r, nq):
    return np.abs(np.asarray(a) - np.asarray(r)) * 2.0 ** (nq / 2)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_3m"])
@pytest.mark.parametrize("L,d,seed,nb", [(2, 8, 0, 16), (4, 16, 1, 48), (4, 24, 2, 48)])
def test_square_small_vs_state_vector(ps, prec, L, d, seed, nb):
    c = rqcgen.generate(L, L, d, seed)
    bits = rqcgen.all_bitstrings(L * L) if L == 2 else rqcgen.bitstrings(L, L, seed, nb)
    ref = sv.amplitudes(sv.run(c), bits)
    pl = ps.Plan(ps.Peps(c), prec=prec, sweep=3)
    assert pl.stats()["sweep"] == 3
    a = pl.amplitudes(bits)
    e = _eps_rms(a, ref, L * L)
    say(f"square {L}x{L} d{d} {prec}: max eps_rms {e.max():.2e}")
    assert e.max() <= AMP_BAR[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32_3m"])
@pytest.mark.parametrize("lv,lh,d,seed", [(3, 3, 8, 0), (3, 5, 16, 1), (5, 4, 16, 2), (2, 6, 13, 3)])
def test_square_odd_and_rectangular_vs_state_vector(ps, prec, lv, lh, d, seed):
    """Uneven quadrants: odd sides (eqs. S11-S12) and rectangular lattices."""
    c = rqcgen.generate(lv, lh, d, seed)
    bits = rqcgen.all_bitstrings(9) if lv * lh == 9 else rqcgen.bitstrings(lv, lh, seed, 40)
    ref = sv.amplitudes(sv.run(c), bits)
    a = ps.Plan(ps.Peps(c), prec=prec, sweep=3, max_batch=len(bits)).amplitudes(bits)
    e = _eps_rms(a, ref, lv * lh)
    say(f"square {lv}x{lh} d{d} {prec}: max eps_rms {e.max():.2e}")
    assert e.max() <= AMP_BAR[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32_3m"])
def test_square_5x5_d32_golden(ps, prec):
    """5x5 (1+32+1), 256 bitstrings: the odd partition against the state vector."""
    with open(os.path.join(HERE, "golden", "rqc_5x5_d32_s0.json")) as f:
        g = json.load(f)
    c = rqcgen.generate(5, 5, 32, 0)
    assert c.sha256() == g["sha256"]
    bits = np.array(g["bits"], dtype=np.uint8)
    ref = np.array(g["amps_re"]) + 1j * np.array(g["amps_im"])
    a = ps.Plan(ps.Peps(c), prec=prec, sweep=3, max_batch=len(bits)).amplitudes(bits)
    e = _eps_rms(a, ref, 25)
    say(f"square 5x5 d32 {prec}: max eps_rms {e.max():.2e}")
    assert e.max() <= AMP_BAR[prec]


def test_square_6x6_d16_vs_oracle_and_row_scheme(ps):
    c = rqcgen.generate(6, 6, 16, 3)
    bits = rqcgen.bitstrings(6, 6, 3, 12)
    ref = opeps.amplitudes(opeps.build(c), bits)
    P = ps.Peps(c)
    sq = ps.Plan(P, prec="fp64", sweep=3).amplitudes(bits)
    row = ps.Plan(P, prec="fp64", max_batch=len(bits)).amplitudes(bits)
    assert np.max(np.abs(sq - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(sq - row)) <= 1e-12 * np.max(np.abs(ref))
    a3 = ps.Plan(P, prec="fp32_3m", sweep=3).amplitudes(bits)
    assert _eps_rms(a3, ref, 36).max() <= AMP_BAR["fp32_3m"]


def test_square_general_gates(ps):
    """Arbitrary one- and two-qubit gates (bond dimensions up to 4 per gate,
    uneven bonds) through the square partition."""
    c = rqcgen.generate_general(4, 4, 3, 7, "U2")
    bits = rqcgen.bitstrings(4, 4, 7, 24)
    ref = sv.amplitudes(sv.run(c), bits)
    for prec, bar in (("fp64", 1e-10), ("fp32_3m", 1e-5)):
        a = ps.Plan(ps.Peps(c), prec=prec, sweep=3, max_batch=len(bits)).amplitudes(bits)
        assert _eps_rms(a, ref, 16).max() <= bar, prec


def test_square_duplicates_and_order(ps):
    """Bitstrings in any order, with repeats, sharing some quadrants."""
    c = rqcgen.generate(4, 4, 16, 5)
    base = rqcgen.bitstrings(4, 4, 5, 6)
    bits = np.concatenate([base, base[::-1], base[:2]])
    bits[3, 15] ^= 1                     # differs from base[3] in the lower-right quadrant only
    ref = sv.amplitudes(sv.run(c), bits)
    P = ps.Peps(c)
    a = ps.Plan(P, prec="fp64", sweep=3).amplitudes(bits)            # one lower-left pattern per pass
    assert np.max(np.abs(a - ref)) <= 1e-12 * np.max(np.abs(ref))
    a2 = ps.Plan(P, prec="fp64", sweep=3, max_batch=len(bits)).amplitudes(bits)   # several per pass
    assert np.max(np.abs(a2 - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["fp32_3m", "fp64"])
def test_square_6x6_d40_vs_golden(ps, prec):
    with open(os.path.join(HERE, "golden", "rqc_6x6_d40_s0.json")) as f:
        g = json.load(f)
    c = rqcgen.generate(6, 6, 40, 0)
    assert c.sha256() == g["sha256"]
    bits = np.array(g["bits"], dtype=np.uint8)
    ref = np.array(g["amps_re"]) + 1j * np.array(g["amps_im"])
    # FP32: two Y tensors fit the budget (both lower-left patterns in one pass); FP64: one per pass
    pl = ps.Plan(ps.Peps(c), prec=prec, sweep=3, max_batch=len(bits),
                 mem_budget=(64 if prec != "fp64" else 120) << 30)
    say(f"square 6x6 d40 {prec}: workspace {pl.stats()['workspace_bytes'] / 2**30:.1f} GiB")
    a = pl.amplitudes(bits)
    rel = np.abs(a - ref) / np.abs(ref)
    say(f"square 6x6 d40 {prec}: max eps_rel {rel.max():.2e}")
    assert rel.max() <= (1e-10 if prec == "fp64" else 1e-5)


def _shared_batch(lv, lh, seed, n):
    """n random bitstrings, then copies of the first 30 with the last qubit
    (a lower-right site) flipped (same upper half and lower-left quadrant),
    then repeats of the first 5: 35 + n bitstrings."""
    base = rqcgen.bitstrings(lv, lh, seed, n)
    flip = base[:30].copy()
    flip[:, lv * lh - 1] ^= 1
    return np.concatenate([base, flip, base[:5]])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_3m"])
@pytest.mark.parametrize("lv,lh,d,seed", [(3, 3, 8, 0), (4, 4, 16, 1), (3, 5, 16, 2), (5, 4, 16, 3),
                                          (2, 6, 13, 4), (4, 5, 16, 5)])
def test_square_chunks_match_one_by_one(ps, prec, lv, lh, d, seed):
    """The batched form (a chunk of up to 32 bitstrings, each quadrant's
    distinct patterns as the node index of one set of launches) against the
    one-by-one form (max_batch 1): the same launches per tensor, so the same
    amplitudes bit for bit; 75 bitstrings = three chunks, the last one ragged,
    with shared halves and repeats; and the state vector within the bar."""
    c = rqcgen.generate(lv, lh, d, seed)
    bits = _shared_batch(lv, lh, seed, 40)
    P = ps.Peps(c)
    one = ps.Plan(P, prec=prec, sweep=3, max_batch=1)
    chunked = ps.Plan(P, prec=prec, sweep=3, max_batch=len(bits))
    assert chunked.stats()["workspace_bytes"] > one.stats()["workspace_bytes"]
    a1 = one.amplitudes(bits)
    chunked.profile_start()
    a2 = chunked.amplitudes(bits)
    prof = chunked.profile_read()
    chunked.profile_stop()
    assert np.array_equal(a1, a2), np.max(np.abs(a1 - a2))
    # each quadrant's sites once per chunk (3 chunks), the upper and
    # lower-left ones only where a chunk cannot reuse the previous T / Y
    n_lr = (lv - lv // 2) * (lh - lh // 2)
    assert lv * lh + 2 * n_lr <= prof["first_site"]["launches"] <= 3 * lv * lh, prof["first_site"]
    ref = sv.amplitudes(sv.run(c), bits)
    e = _eps_rms(a2, ref, lv * lh)
    say(f"square chunks {lv}x{lh} d{d} {prec}: bitwise equal to one by one, max eps_rms {e.max():.2e}")
    assert e.max() <= AMP_BAR[prec]


def test_square_chunk_budget_and_repeat_calls(ps):
    """A budget too small for a chunk of 8 gives the one-by-one form; a
    chunked plan called twice in a row (the second call smaller) repeats its
    results exactly."""
    c = rqcgen.generate(5, 5, 24, 6)
    bits = _shared_batch(5, 5, 6, 20)
    P = ps.Peps(c)
    full = ps.Plan(P, prec="fp32_3m", sweep=3, max_batch=len(bits))
    one = ps.Plan(P, prec="fp32_3m", sweep=3, max_batch=1)
    small = ps.Plan(P, prec="fp32_3m", sweep=3, max_batch=len(bits),
                    mem_budget=one.stats()["workspace_bytes"] + (1 << 20))
    assert small.stats()["workspace_bytes"] == one.stats()["workspace_bytes"]
    a = full.amplitudes(bits)
    assert np.array_equal(a, small.amplitudes(bits))
    assert np.array_equal(full.amplitudes(bits[7:20]), a[7:20])
    assert np.array_equal(full.amplitudes(bits), a)


@pytest.mark.parametrize("prec", ["fp64", "fp32_3m"])
def test_square_fast_sampling_reuse(ps, prec):
    """Bitstrings that differ only in the lower-right quadrant (the
    fast-sampling case): the first chunk contracts T and Y, the next two
    reuse them (2 join launches in all, lower-right sites only after the
    first chunk); bit for bit equal to one by one, and the state vector."""
    c = rqcgen.generate(4, 5, 16, 7)
    base = rqcgen.bitstrings(4, 5, 7, 1)[0]
    lr = [12, 13, 14, 17, 18, 19]              # rows 2-3, columns 2-4
    vals = rqcgen.all_bitstrings(6)
    bits = np.repeat(base[None, :], 75, axis=0)
    bits[:64, lr] = vals
    bits[64:, lr] = vals[5:16]                 # repeats
    P = ps.Peps(c)
    one = ps.Plan(P, prec=prec, sweep=3, max_batch=1)
    chunked = ps.Plan(P, prec=prec, sweep=3, max_batch=len(bits))
    chunked.profile_start()
    a2 = chunked.amplitudes(bits)
    prof = chunked.profile_read()
    chunked.profile_stop()
    assert np.array_equal(one.amplitudes(bits), a2)
    assert prof["interior_site"]["launches"] == 2, prof["interior_site"]
    assert prof["first_site"]["launches"] == 20 + 2 * 6, prof["first_site"]
    ref = sv.amplitudes(sv.run(c), bits)
    e = _eps_rms(a2, ref, 20)
    say(f"square fast sampling 4x5 d16 {prec}: max eps_rms {e.max():.2e}")
    assert e.max() <= AMP_BAR[prec]


def test_square_empty_and_single(ps):
    """No bitstrings: nothing to do, an empty result; one bitstring in a
    chunked plan equals the one-by-one form."""
    c = rqcgen.generate(4, 4, 16, 9)
    P = ps.Peps(c)
    for mb in (1, 64):
        pl = ps.Plan(P, prec="fp32_3m", sweep=3, max_batch=mb)
        assert pl.amplitudes(np.zeros((0, 16), dtype=np.uint8)).size == 0
    b = rqcgen.bitstrings(4, 4, 9, 1)
    a1 = ps.Plan(P, prec="fp32_3m", sweep=3, max_batch=1).amplitudes(b)
    a2 = ps.Plan(P, prec="fp32_3m", sweep=3, max_batch=64).amplitudes(b)
    assert np.array_equal(a1, a2)


def test_square_split_accumulation(ps):
    """PSIM_PLAN_SPLIT_ACC in the square partition (quadrant sites and joins
    in the split kernels): on 6x6 (1+40+1) the amplitudes differ from the
    unsplit plan's (the split kernels ran) and stay within 1e-5 of the golden
    values; on 4x5 the chunked form equals the one-by-one form bit for bit."""
    with open(os.path.join(HERE, "golden", "rqc_6x6_d40_s0.json")) as f:
        g = json.load(f)
    c = rqcgen.generate(6, 6, 40, 0)
    bits = np.array(g["bits"], dtype=np.uint8)
    ref = np.array(g["amps_re"]) + 1j * np.array(g["amps_im"])
    P = ps.Peps(c)
    kw = dict(prec="fp32_3m", sweep=3, max_batch=len(bits), mem_budget=64 << 30)
    a0 = ps.Plan(P, **kw).amplitudes(bits)
    a1 = ps.Plan(P, split_acc=True, **kw).amplitudes(bits)
    r0, r1 = (np.abs(a - ref) / np.abs(ref) for a in (a0, a1))
    say(f"square 6x6 d40 fp32_3m: max eps_rel {r0.max():.2e} unsplit, {r1.max():.2e} split")
    assert not np.array_equal(a0, a1)
    assert r1.max() <= 1e-5
    c = rqcgen.generate(4, 5, 16, 5)
    b = _shared_batch(4, 5, 5, 40)
    P = ps.Peps(c)
    one = ps.Plan(P, prec="fp32", sweep=3, max_batch=1, split_acc=True).amplitudes(b)
    chunked = ps.Plan(P, prec="fp32", sweep=3, max_batch=len(b), split_acc=True).amplitudes(b)
    assert np.array_equal(one, chunked)
    e = _eps_rms(chunked, sv.amplitudes(sv.run(c), b), 20)
    assert e.max() <= AMP_BAR["fp32"]
