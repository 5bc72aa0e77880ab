"""Why the library reports measured errors instead of an a-priori bound.

A first-order rounding bound for a contraction computed in floating point is
gamma * N_abs(tau), with N_abs the same network contracted with |E_n| (the
entrywise absolute values of the projected site tensors, eq. 7) and gamma of
order (number of accumulated terms) * unit roundoff.  For random circuits
N_abs / |<tau|psi>| grows exponentially with lattice size and depth (no
cancellation is left in the absolute values), so the relative bound exceeds 1
long before the 6x6 (1+40+1) workload; this test pins that growth on small
lattices with the oracle."""
import numpy as np

import rqcgen
from oracle import peps as op


def _ratio(lv, lh, d, seed, b):
    c = rqcgen.generate(lv, lh, d, seed)
    P = op.build(c)
    bits = rqcgen.bitstrings(lv, lh, seed, b + 1)[b]
    sites = op.projected_sites(P, bits)
    order = op.site_order(lv, lh, "rows")
    a = op.contract_sites(sites, order).a.reshape(-1)[0]
    absd = {k: op.LT(np.abs(v.a), v.labels) for k, v in sites.items()}
    n = op.contract_sites(absd, order).a.reshape(-1)[0]
    assert n.imag == 0 and n.real >= abs(a)      # triangle inequality
    return n.real / abs(a)


def test_absolute_value_contraction_outgrows_fp32():
    u32 = 2.0 ** -24
    small = _ratio(3, 3, 8, 0, 0)
    mid = _ratio(4, 5, 24, 0, 0)
    big = _ratio(5, 5, 24, 0, 0)
    assert small < 1e3 < mid < big
    # already at 5x5 (1+24+1) the bound's prefactor alone exceeds 1 / u32
    assert big * u32 > 1.0
