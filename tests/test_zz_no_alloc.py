"""psim_amplitudes_static (the allocation-free entry point) against
psim_amplitudes on the same plans, through the C ABI: the same amplitudes bit
for bit, within the oracle bar, on two calls in a row (the second smaller),
and a plan too large for the static workspace refused with outputs untouched."""
import ctypes
import json
import os

import numpy as np
import pytest

import rqcgen
from parity_bars import BAR, report

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ps():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1905_08394_amd as ps
    ps.lib()
    return ps


def _static(ps, plan, bits, stream=None):
    import torch
    bits = np.ascontiguousarray(bits, dtype=np.uint8)
    out = np.zeros(2 * len(bits))
    st = torch.cuda.current_stream().cuda_stream if stream is None else stream
    status = ps.lib().psim_amplitudes_static(plan._h, bits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), len(bits),
                                             ctypes.c_void_p(st), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             None)
    return status, out[0::2] + 1j * out[1::2]


def _golden(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        g = json.load(f)
    return np.array(g["bits"], dtype=np.uint8), np.array(g["amps_re"]) + 1j * np.array(g["amps_im"])


@pytest.mark.parametrize("lv,lh,d,prec,sweep,golden", [
    (4, 5, 24, "fp32_3m", 0, "rqc_4x5_d24_s0.json"),
    (3, 3, 8, "fp64", 0, "rqc_3x3_d8_s0.json"),
    (3, 3, 8, "fp32", 3, "rqc_3x3_d8_s0.json"),
    (4, 5, 24, "fp32_3ms", 0, "rqc_4x5_d24_s0.json"),   # split accumulation
])
def test_static_matches_workspace_entry(ps, lv, lh, d, prec, sweep, golden):
    bits, ref = _golden(golden)
    c = rqcgen.generate(lv, lh, d, 0)
    P = ps.Peps(c)
    split = prec == "fp32_3ms"
    plan = ps.Plan(P, prec="fp32_3m" if split else prec, max_batch=len(bits), sweep=sweep, split_acc=split)
    assert plan.stats()["workspace_bytes"] <= 64 << 20
    n = lv * lh
    for sel in (slice(None), slice(3, 3 + max(1, len(bits) // 4))):   # second call smaller
        b = bits[sel]
        print(f"static {lv}x{lh} d{d} {prec} sweep {sweep}: {len(b)} bitstrings", flush=True)
        st, a = _static(ps, plan, b)
        assert st == ps.PSIM_OK, ps.lib().psim_last_error()
        want = plan.amplitudes(b)
        assert np.array_equal(a, want)
        assert report(f"static {lv}x{lh} {prec}", a, ref[sel], n) <= BAR[prec]
    plan.close()
    P.close()


def test_static_refuses_large_plan(ps):
    c = rqcgen.generate(5, 5, 32, 0)
    P = ps.Peps(c)
    plan = ps.Plan(P, prec="fp32_3m", max_batch=16, mem_budget=48 << 30)
    assert plan.stats()["workspace_bytes"] > 64 << 20
    bits = rqcgen.bitstrings(5, 5, 0, 2)
    import torch
    out = np.full(4, 7.0)
    status = ps.lib().psim_amplitudes_static(plan._h, np.ascontiguousarray(bits).ctypes.data_as(
        ctypes.POINTER(ctypes.c_uint8)), 2, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None)
    assert status == ps.PSIM_EINVAL
    assert b"static workspace" in ps.lib().psim_last_error()
    assert np.all(out == 7.0)
    plan.close()
    P.close()
