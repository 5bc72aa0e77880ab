"""Write the golden amplitudes the GPU parity tests compare against.

Every value here comes from the CPU oracle (package `oracle`) on inputs from
the seeded generator `rqcgen`; nothing is read from the GPU library.

  python tests/golden/make_golden.py            # 3x3, 4x5, 5x5 (minutes)
  python tests/golden/make_golden.py --big      # also 6x6 d40 (about an hour, ~34 GiB RAM)
  python tests/golden/make_golden.py --only-big --base 1   # 6x6 d40, second base bitstring
  python tests/golden/make_golden.py --rows6    # 6x6 d40 base 0 again, by the row scheme (about 11 h here)
  python tests/golden/make_golden.py --halves6  # 6x6 d40 base amplitude by the left/right halves (about 1 h)

Files: rqc_<lv>x<lh>_d<d>_s<seed>.json with the circuit hash, the bitstrings
and the FP64 amplitudes.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import rqcgen  # noqa: E402
from oracle import peps, statevector as sv, stats  # noqa: E402


def _write(name, circuit, bits, amps, method, extra=None):
    d = {
        "lv": circuit.lv, "lh": circuit.lh, "depth": circuit.depth, "seed": circuit.seed,
        "sha256": circuit.sha256(), "method": method,
        "bits": np.asarray(bits, dtype=int).tolist(),
        "amps_re": [float(a.real) for a in amps], "amps_im": [float(a.imag) for a in amps],
    }
    if extra:
        d.update(extra)
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(d, f)
    print("wrote", name, flush=True)


def small():
    c = rqcgen.generate(3, 3, 8, 0)
    bits = rqcgen.all_bitstrings(9)
    _write("rqc_3x3_d8_s0.json", c, bits, sv.amplitudes(sv.run(c), bits), "statevector")

    for seed in range(8):
        c = rqcgen.generate(4, 5, 24, seed)
        bits = rqcgen.bitstrings(4, 5, seed, 64)
        _write(f"rqc_4x5_d24_s{seed}.json", c, bits, sv.amplitudes(sv.run(c), bits), "statevector")

    c = rqcgen.generate(5, 5, 32, 0)
    t = time.time()
    psi = sv.run(c)
    bits = rqcgen.bitstrings(5, 5, 0, 256)
    amps = sv.amplitudes(psi, bits)
    pt = stats.porter_thomas_summary(stats.scaled_probabilities(psi.reshape(-1), 25))
    print("5x5 state vector", time.time() - t, pt, flush=True)
    del psi
    # cross-check a few with the PEPS row scheme (an independent computation)
    P = peps.build(c)
    chk = peps.amplitudes(P, bits[:4])
    assert np.max(np.abs(chk - amps[:4])) < 1e-12 * np.max(np.abs(amps))
    _write("rqc_5x5_d32_s0.json", c, bits, amps, "statevector", {"porter_thomas_full": pt})


def big(base_index=0):
    """Base bitstring `base_index` of the seeded stream and its 16 last-row
    variants (columns 2-5), by the sliced square partition (eqs. S9-S10)."""
    c = rqcgen.generate(6, 6, 40, 0)
    base = rqcgen.bitstrings(6, 6, 0, base_index + 1)[base_index]
    cols = [2, 3, 4, 5]
    var = rqcgen.last_row_variants(base, 6, 6, cols)     # variant i: cols bits = bits of i
    left = var[[0, 8]]                                    # column 2 = 0 / 1 (bottom-left quadrant)
    right = var[list(range(8))]                           # columns 3..5 = 000..111 (bottom-right)
    t = time.time()
    P = peps.build(c)
    res = peps.quadrant_amplitudes_sliced(P, base, left, right,
                                          log=lambda s: print(f"[{time.time() - t:7.0f}s] {s}", flush=True))
    amps = res.reshape(-1)                                # i * 8 + j == variant index
    name = "rqc_6x6_d40_s0.json" if base_index == 0 else f"rqc_6x6_d40_s0_b{base_index}.json"
    _write(name, c, var, amps, "peps-square-partition-sliced",
           {"base_index": int(next(i for i in range(16) if np.array_equal(var[i], base))),
            "variant_cols": cols, "stream_index": base_index, "seconds": time.time() - t})


def rows6():
    """The 16 amplitudes of the base-0 6x6 (1+40+1) batch again, by the row
    scheme (supplement S-II) with cut loops: an order independent of the
    square partition that wrote rqc_6x6_d40_s0.json (several hours on 8 cores,
    ~34 GiB RAM)."""
    c = rqcgen.generate(6, 6, 40, 0)
    base = rqcgen.bitstrings(6, 6, 0, 1)[0]
    var = rqcgen.last_row_variants(base, 6, 6, [2, 3, 4, 5])
    t = time.time()
    P = peps.build(c)
    amps = peps.row_amplitudes_sliced(P, base, var,
                                      log=lambda s: print(f"[{time.time() - t:7.0f}s] {s}", flush=True))
    _write("rqc_6x6_d40_s0_rows.json", c, var, amps, "peps-row-scheme-sliced",
           {"variant_cols": [2, 3, 4, 5], "seconds": time.time() - t})


def halves6():
    """The base amplitude of the base-0 6x6 (1+40+1) batch again, by the
    square partition grouped into left and right halves (a contraction order
    and cut loops other than those that wrote rqc_6x6_d40_s0.json; about an
    hour on 8 cores, ~34 GiB RAM)."""
    c = rqcgen.generate(6, 6, 40, 0)
    base = rqcgen.bitstrings(6, 6, 0, 1)[0]
    t = time.time()
    P = peps.build(c)
    amp = peps.halves_amplitude_sliced(P, base, log=lambda s: print(f"[{time.time() - t:7.0f}s] {s}", flush=True))
    _write("rqc_6x6_d40_s0_halves.json", c, base[None, :], np.array([amp]), "peps-square-partition-halves-sliced",
           {"seconds": time.time() - t})


def fig2():
    """8x8 (1+25+1), the lattice of the paper's Porter-Thomas figure: eight
    amplitudes by the oracle's row scheme (largest tensor 8^8 x 16 elements)."""
    c = rqcgen.generate(8, 8, 25, 0)
    bits = rqcgen.bitstrings(8, 8, 0, 8)
    t = time.time()
    P = peps.build(c)
    amps = []
    for i, b in enumerate(bits):
        amps.append(peps.amplitude(P, b, "rows"))
        print(f"[{time.time() - t:6.0f}s] 8x8 amplitude {i + 1}/8", flush=True)
    # an independent order for the first two
    for i in range(2):
        a2 = peps.amplitude(P, bits[i], "rows_bu")
        assert abs(a2 - amps[i]) <= 1e-12 * abs(amps[i]), (a2, amps[i])
    _write("rqc_8x8_d25_s0.json", c, bits, np.array(amps), "peps-row-scheme", {"seconds": time.time() - t})


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--big", action="store_true")
    ap.add_argument("--only-big", action="store_true")
    ap.add_argument("--fig2", action="store_true", help="8x8 (1+25+1) amplitudes")
    ap.add_argument("--rows6", action="store_true", help="6x6 d40 base-0 batch by the sliced row scheme")
    ap.add_argument("--halves6", action="store_true", help="6x6 d40 base amplitude by the left/right halves")
    ap.add_argument("--base", type=int, default=0, help="--big: index of the base bitstring in the stream")
    a = ap.parse_args()
    if a.halves6:
        halves6()
    elif a.rows6:
        rows6()
    elif a.fig2:
        fig2()
    elif not a.only_big:
        small()
    if a.big or a.only_big:
        big(a.base)
