"""Porter-Thomas statistics of deep random circuits (Fig. 2 of the paper)."""
import numpy as np
import pytest

import rqcgen
from oracle import statevector as sv
from oracle import stats


def test_pt_closed_forms_on_exponential_samples():
    rng = np.random.default_rng(0)
    x = rng.exponential(size=200000)
    s = stats.porter_thomas_summary(x)
    assert abs(s["mean"] - 1) < 0.01
    assert abs(s["second_moment"] - 2) < 0.05
    assert abs(s["mean_neg_log"] - stats.EULER_GAMMA) < 0.01
    y = np.linspace(-8, 3, 20001)
    assert abs(np.trapezoid(stats.log_pt_density(y), y) - 1) < 1e-3


def _summary(lv, lh, d, seed=0):
    c = rqcgen.generate(lv, lh, d, seed)
    return stats.porter_thomas_summary(stats.scaled_probabilities(sv.run(c).reshape(-1), lv * lh))


def test_4x5_approaches_porter_thomas_with_depth():
    s24, s40, s64 = (_summary(4, 5, d) for d in (24, 40, 64))
    for s in (s24, s40, s64):
        assert abs(s["mean"] - 1) < 1e-10          # normalisation, exact
    # depth (1+24+1) on 4x5 is not yet fully Porter-Thomas; deeper circuits converge
    assert s24["second_moment"] > s40["second_moment"] > s64["second_moment"]
    assert abs(s64["second_moment"] - 2) < 0.02
    assert abs(s64["mean_neg_log"] - stats.EULER_GAMMA) < 0.01
    assert s64["ks_pvalue"] > 0.01


def test_shallow_circuit_is_not_porter_thomas():
    c = rqcgen.generate(4, 5, 4, 0)
    x = stats.scaled_probabilities(sv.run(c).reshape(-1), 20)
    s = stats.porter_thomas_summary(x)
    assert abs(s["second_moment"] - 2) > 0.1 or s["ks_statistic"] > 0.05
