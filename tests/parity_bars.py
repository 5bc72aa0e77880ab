"""Parity bars of the GPU amplitude tests, stated before the runs they apply to.

For an amplitude a on N qubits against the FP64 oracle value r, with
x = 2^N |r|^2 (the scaled probability; Porter-Thomas: x ~ Exp(1)):

  eps_rel   = |a - r| / |r|                          per amplitude (the target's measure)
  eps_rms   = |a - r| * 2^(N/2)                       relative to the RMS amplitude
  eps_floor = |a - r| / max(|r|, sqrt(X_MIN) 2^(-N/2))

The bar is eps_floor <= BAR[prec] on every amplitude.  For x >= X_MIN = 0.1
(about 90 % of a Porter-Thomas sample) this is exactly eps_rel <= BAR; in the
tail x < 0.1 it caps the absolute error at BAR * sqrt(0.1) * 2^(-N/2), i.e.
eps_rms <= 3.2e-6 for FP32.  The floor exists because rounding in FP32 leaves
an absolute error of a few 1e-6 times the RMS amplitude whatever the size of
the amplitude, so eps_rel grows as x^(-1/2) into the tail; exact zeros (small
symmetric circuits) would make eps_rel undefined.

  FP64                        1e-10
  FP32 4M, 3M (split or not)  1e-5
  BF16x3                      1e-3
"""
import numpy as np

X_MIN = 0.1
BAR = {"fp64": 1e-10, "fp32": 1e-5, "fp32s": 1e-5, "fp32_3m": 1e-5, "fp32_3ms": 1e-5, "bf16x3": 1e-3}

# Measured against that bar on the 32 amplitudes of 6x6 (1+40+1): the FP32
# forms WITHOUT split accumulation miss it (worst eps_rel 1.16e-5 for 4M,
# 1.25e-5 for 3M, both at x >= 0.1; the sequential FP32 sums over K = 1024
# and over the v values of a pass grow with the lattice), the split forms meet
# it (3.4e-6 4M, 5.5e-6 3M), so the split 3M form is the default and the one
# the 1e-5 target is claimed for.  The unsplit forms are held at 6x6 to the
# regression bar below, which is not the target.
BAR_C4_UNSPLIT = 2e-5


def measures(a, r, n):
    """(eps_rel, eps_rms, eps_floor, x) of every amplitude."""
    a, r = np.asarray(a), np.asarray(r)
    d = np.abs(a - r)
    x = np.abs(r) ** 2 * 2.0 ** n
    floor = np.sqrt(X_MIN) * 2.0 ** (-n / 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(np.abs(r) > 0, d / np.abs(r), np.inf)
    return rel, d * 2.0 ** (n / 2), d / np.maximum(np.abs(r), floor), x


def report(tag, a, r, n):
    """One line: worst eps_floor with its eps_rel and x, the worst eps_rel
    among x >= X_MIN, the median eps_rel; returns the worst eps_floor."""
    rel, rms, fl, x = measures(a, r, n)
    i = int(np.argmax(fl))
    big = x >= X_MIN
    worst_big = float(np.max(rel[big])) if np.any(big) else 0.0
    print(f"{tag}: {len(fl)} amplitudes, worst eps_floor {fl[i]:.3e} (eps_rel {rel[i]:.3e} at x = {x[i]:.3g}); "
          f"max eps_rel over x >= {X_MIN} {worst_big:.3e}; max eps_rms {np.max(rms):.3e}; "
          f"median eps_rel {np.median(rel[np.isfinite(rel)]):.3e}; min x {np.min(x):.3g}", flush=True)
    return float(fl[i])
