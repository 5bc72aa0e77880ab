"""GPU parity of grouped (mixed-circuit) launches: several plans, different
lattices and depths, contracted in one interleaved sweep (psim_group).

Each plan's grouped result must equal its own psim_amplitudes result bit for
bit (the merged launches run the same kernel body on the same tiles), and the
oracle within the precision's bar (eps_rms, as in the single-plan tests)."""
import ctypes
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
AMP_BAR = {"fp64": 1e-10, "fp32": 1e-5, "fp32_3m": 1e-5, "bf16x3": 1e-3, "fp32s": 1e-5, "fp32_3ms": 1e-5}
# fp32s / fp32_3ms: FP32 4M / 3M plans with split accumulation
SPLIT = {"fp32s": "fp32", "fp32_3ms": "fp32_3m"}

# (lv, lh, depth, seed, bitstrings): uneven lattices, depths and bond sizes
MIX = [(3, 3, 8, 0, 32), (4, 5, 24, 1, 64), (3, 4, 13, 2, 24), (4, 4, 24, 5, 40),
       (2, 6, 16, 4, 16), (5, 5, 24, 6, 48), (6, 6, 16, 3, 16)]


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


_REF = {}


def _reference(c, bits):
    """FP64 oracle: state vector up to 20 qubits, the oracle's PEPS row scheme above
    (pinned to the state vector by the oracle tests)."""
    key = (c.sha256(), bits.tobytes())
    if key not in _REF:
        if c.lv * c.lh <= 20:
            _REF[key] = sv.amplitudes(sv.run(c), bits)
        else:
            _REF[key] = opeps.amplitudes(opeps.build(c), bits)
    return _REF[key]


def _mix():
    out = []
    for lv, lh, d, seed, n in MIX:
        c = rqcgen.generate(lv, lh, d, seed)
        out.append((c, rqcgen.bitstrings(lv, lh, seed, n)))
    return out


def _check(ps, mix, precs, max_batch=None):
    plans = []
    for k, (c, bits) in enumerate(mix):
        mb = len(bits) if max_batch is None else max_batch[k]
        p = precs[k]
        plans.append(ps.Plan(ps.Peps(c), prec=SPLIT.get(p, p), max_batch=mb, split_acc=p in SPLIT))
    single = [p.amplitudes(b) for p, (c, b) in zip(plans, mix)]
    g = ps.Group(plans)
    grouped = g.amplitudes([b for c, b in mix])
    for k, ((c, bits), a, s) in enumerate(zip(mix, grouped, single)):
        assert np.array_equal(a, s), (k, c.lv, c.lh, c.depth, np.max(np.abs(a - s)))
        r = _reference(c, bits)
        e_rms = np.abs(a - r) * 2.0 ** (c.lv * c.lh / 2)
        say(f"group {precs[k]} {c.lv}x{c.lh} d{c.depth}: max eps_rms {e_rms.max():.2e}")
        assert e_rms.max() <= AMP_BAR[precs[k]], (k, e_rms.max())
    st = g.stats()
    g.close()
    return st


@pytest.mark.parametrize("prec", ["fp32", "fp32_3m"])
def test_group_matches_single_and_oracle(ps, prec):
    mix = _mix()
    say(f"group test {prec}: {len(mix)} circuits")
    st = _check(ps, mix, [prec] * len(mix))
    assert st["n_plans"] == len(mix)
    assert st["grouped_launches"] > 0


def test_group_mixed_precisions_and_passes(ps):
    """FP64 / BF16x3 plans (launched one by one) next to FP32 ones, and plans
    whose batches need several passes (max_batch below the bitstring count)."""
    mix = _mix()
    precs = ["fp64", "fp32", "bf16x3", "fp32_3m", "fp32", "fp32", "fp32_3m"]
    mb = [32, 16, 24, 7, 16, 48, 5]
    say("group test mixed precisions / passes")
    st = _check(ps, mix, precs, mb)
    assert st["grouped_launches"] > 0


def test_group_with_split_accumulation_plans(ps):
    """Split-accumulation plans (launched one by one) in a group with
    unsplit FP32 plans, whose launches are still merged."""
    mix = _mix()
    precs = ["fp32_3ms", "fp32", "fp32s", "fp32_3m", "fp32_3ms", "fp32", "fp32_3m"]
    say("group test with split-accumulation plans")
    st = _check(ps, mix, precs)
    assert st["grouped_launches"] > 0


def test_group_repeat_and_empty(ps):
    """Two calls in a row (the second with fewer bitstrings and one plan left
    empty) agree with the single-plan path."""
    mix = _mix()[:4]
    plans = [ps.Plan(ps.Peps(c), prec="fp32", max_batch=len(b)) for c, b in mix]
    g = ps.Group(plans)
    first = g.amplitudes([b for c, b in mix])
    for p, (c, b), a in zip(plans, mix, first):
        assert np.array_equal(a, p.amplitudes(b))
    second_bits = [b[: max(1, len(b) // 3)] for c, b in mix]
    second_bits[2] = second_bits[2][:0]
    second = g.amplitudes(second_bits)
    for k, (p, b, a) in enumerate(zip(plans, second_bits, second)):
        if len(b) == 0:
            assert a.size == 0
            continue
        assert np.array_equal(a, p.amplitudes(b)), k
    g.close()


def test_group_errors(ps):
    mix = _mix()[:2]
    plans = [ps.Plan(ps.Peps(c), prec="fp32", max_batch=len(b)) for c, b in mix]
    g = ps.Group(plans)
    L = ps.lib()
    # overlapping workspaces
    ws = plans[1].workspace()
    bs = [np.ascontiguousarray(b, dtype=np.uint8) for c, b in mix]
    outs = [np.zeros(2 * len(b)) for b in bs]
    PU8 = ctypes.POINTER(ctypes.c_uint8)
    PD = ctypes.POINTER(ctypes.c_double)
    c_bits = (PU8 * 2)(*[b.ctypes.data_as(PU8) for b in bs])
    c_n = (ctypes.c_size_t * 2)(*[len(b) for b in bs])
    big = max(p.stats()["workspace_bytes"] for p in plans)
    import torch
    shared = torch.empty(big, dtype=torch.uint8, device="cuda:0")
    c_ws = (ctypes.c_void_p * 2)(shared.data_ptr(), shared.data_ptr())
    c_wsb = (ctypes.c_size_t * 2)(big, big)
    c_out = (PD * 2)(*[o.ctypes.data_as(PD) for o in outs])
    st = L.psim_group_amplitudes(g._h, c_bits, c_n, c_ws, c_wsb, None, c_out)
    assert st == ps.PSIM_EINVAL and "overlap" in L.psim_last_error().decode()
    # a bad bit in plan 1: the message names the plan, nothing is written
    bad = bs[1].copy()
    bad[0, 0] = 2
    c_bits[1] = bad.ctypes.data_as(PU8)
    c_ws[1] = ws.data_ptr()
    c_wsb[1] = ws.numel()
    st = L.psim_group_amplitudes(g._h, c_bits, c_n, c_ws, c_wsb, None, c_out)
    assert st == ps.PSIM_EINVAL and "plan 1" in L.psim_last_error().decode()
    assert not outs[0].any() and not outs[1].any()
    g.close()


def test_group_graph_replay(ps):
    """Graph-captured grouped sweeps: first call captures, repeats replay;
    every replay (with eager work and synchronisation in between) equals the
    eager single-plan result bit for bit."""
    import torch
    mix = _mix()[:5]
    eager = [ps.Plan(ps.Peps(c), prec="fp32_3m", max_batch=len(b)) for c, b in mix]
    graphed = [ps.Plan(ps.Peps(c), prec="fp32_3m", max_batch=len(b), graph=True) for c, b in mix]
    g = ps.Group(graphed)
    sets = [[b for c, b in mix],
            [rqcgen.bitstrings(c.lv, c.lh, 100 + k, len(b)) for k, (c, b) in enumerate(mix)]]
    for r, which in enumerate([0, 1, 0, 0, 1]):
        bits = sets[which]
        got = g.amplitudes(bits)
        x = torch.ones(1 << 20, device="cuda:0")       # eager work between replays
        assert float(x.sum()) == float(1 << 20)
        torch.cuda.synchronize()
        for k, (p, b, a) in enumerate(zip(eager, bits, got)):
            assert np.array_equal(a, p.amplitudes(b)), (r, k)
    say(f"group graph replays ok, merged launches {g.stats()['grouped_launches']}")
    g.close()


def test_group_bitwise_with_direct_lds_kernel(ps):
    """5x5 (1+32+1) interior steps (M = 4096, K = N = 256) run the 3M
    direct-to-LDS kernel, on their own and merged with other circuits' steps
    in a grouped launch: the results must agree bit for bit, and with the
    state-vector golden values."""
    with open(os.path.join(HERE, "golden", "rqc_5x5_d32_s0.json")) as f:
        gold = json.load(f)
    bits5 = np.array(gold["bits"][:32], dtype=np.uint8)
    ref5 = (np.array(gold["amps_re"]) + 1j * np.array(gold["amps_im"]))[:32]
    c5 = rqcgen.generate(5, 5, 32, 0)
    assert c5.sha256() == gold["sha256"]
    mix = [(c5, bits5)] + _mix()[:3]
    plans = [ps.Plan(ps.Peps(c), prec="fp32_3m", max_batch=len(b)) for c, b in mix]
    single = [p.amplitudes(b) for p, (c, b) in zip(plans, mix)]
    g = ps.Group(plans)
    grouped = g.amplitudes([b for c, b in mix])
    for k, (a, s) in enumerate(zip(grouped, single)):
        assert np.array_equal(a, s), k
    e_rms = np.abs(single[0] - ref5) * 2.0 ** 12.5
    say(f"5x5 d32 3M (direct-to-LDS) max eps_rms {e_rms.max():.2e}")
    assert e_rms.max() <= AMP_BAR["fp32_3m"]
    g.close()
