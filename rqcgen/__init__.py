"""Seeded random-quantum-circuit and bitstring generator (inputs only).

This module produces the *inputs* of the PEPS amplitude computation: an
ordered list of symbolic gates on an Lv x Lh qubit lattice and the output
bitstrings whose amplitudes are requested.  It holds none of the method's
arithmetic: gates are emitted by name (H, T, SX, SY, CZ) and every consumer
(the CPU oracle, the C library) turns names into matrices on its own.
Random general gates (U1, U2) carry their matrices as plain input data.

Circuit rules (supplement S-I, "Introduction to Random Quantum Circuits"):
a Hadamard layer, then d cycles that each apply CZ on one of eight coupler
patterns and a random gate from {T, sqrt(X), sqrt(Y)} on the other qubits,
then a final Hadamard layer; the depth is written (1+d+1) (main text,
"Quantum Circuit Simulator Based on PEPS" introduction of the depth notation).

The coupler figure (Fig. S1) is not available, so the eight patterns are our
own reading (each one a matching, together a partition of the lattice edges,
so every edge receives exactly one CZ per eight cycles as the chi bound of
eq. (8) assumes):
  horizontal edge (r,c)-(r,c+1) belongs to H_k, k = (c + 2*(r mod 2)) mod 4
  vertical edge   (r,c)-(r+1,c) belongs to V_k, k = (r + 2*(c mod 2)) mod 4
  cycle t >= 1 uses [H0, V0, H1, V1, H2, V2, H3, V3][(t-1) mod 8].
Single-qubit gate choice: a qubit's first gate slot gets T; afterwards one
of the two gates of (SX, SY, T) that differ from its previous gate, picked by
one draw in {0, 1}; qubits are visited row-major inside a cycle.

Qubit n sits at row r = n // Lh, column c = n % Lh; bitstring entry n is the
projected value tau_n of qubit n.
"""
from __future__ import annotations

import hashlib
import json
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

GENERATOR_VERSION = 1
ONE_QUBIT_CHOICES = ("SX", "SY", "T")
KINDS = ("H", "T", "SX", "SY", "CZ", "U1", "U2")


@dataclass
class Gate:
    cycle: int
    kind: str
    q0: int
    q1: int = -1
    m: Optional[List[float]] = None  # U1: 2x2, U2: 4x4 complex row-major as (re, im) pairs

    def to_list(self):
        out = [self.cycle, self.kind, self.q0]
        if self.q1 >= 0:
            out.append(self.q1)
        if self.m is not None:
            if self.q1 < 0:
                out.append(-1)
            out.append([float(x) for x in self.m])
        return out

    @staticmethod
    def from_list(x):
        cycle, kind, q0 = int(x[0]), str(x[1]), int(x[2])
        q1, m = -1, None
        rest = list(x[3:])
        if rest and not isinstance(rest[0], list):
            q1 = int(rest.pop(0))
        if rest:
            m = [float(v) for v in rest.pop(0)]
        return Gate(cycle, kind, q0, q1, m)


@dataclass
class Circuit:
    lv: int
    lh: int
    depth: int
    seed: int
    gates: List[Gate] = field(default_factory=list)
    generator_version: int = GENERATOR_VERSION
    family: str = "rqc"

    @property
    def n_qubits(self) -> int:
        return self.lv * self.lh

    def canonical(self) -> dict:
        return {
            "lv": self.lv, "lh": self.lh, "depth": self.depth, "seed": self.seed,
            "family": self.family, "generator_version": self.generator_version,
            "gates": [g.to_list() for g in self.gates],
        }

    def sha256(self) -> str:
        blob = json.dumps(self.canonical(), sort_keys=True, separators=(",", ":"))
        return hashlib.sha256(blob.encode()).hexdigest()

    def to_json(self) -> str:
        d = self.canonical()
        d["sha256"] = self.sha256()
        return json.dumps(d)

    @staticmethod
    def from_json(s: str) -> "Circuit":
        d = json.loads(s)
        c = Circuit(d["lv"], d["lh"], d["depth"], d["seed"],
                    [Gate.from_list(g) for g in d["gates"]],
                    d.get("generator_version", GENERATOR_VERSION), d.get("family", "rqc"))
        if "sha256" in d and d["sha256"] != c.sha256():
            raise ValueError("circuit.json sha256 mismatch")
        return c


def qubit(lh: int, r: int, c: int) -> int:
    return r * lh + c


def lattice_edges(lv: int, lh: int) -> List[Tuple[int, int]]:
    """All nearest-neighbour pairs (q_left_or_up, q_right_or_down)."""
    e = []
    for r in range(lv):
        for c in range(lh - 1):
            e.append((qubit(lh, r, c), qubit(lh, r, c + 1)))
    for r in range(lv - 1):
        for c in range(lh):
            e.append((qubit(lh, r, c), qubit(lh, r + 1, c)))
    return e


def coupler_pattern(lv: int, lh: int, p: int) -> List[Tuple[int, int]]:
    """Edges of pattern p in cycle order [H0, V0, H1, V1, H2, V2, H3, V3]."""
    k, vertical = p // 2, p % 2 == 1
    out = []
    if not vertical:
        for r in range(lv):
            for c in range(lh - 1):
                if (c + 2 * (r % 2)) % 4 == k:
                    out.append((qubit(lh, r, c), qubit(lh, r, c + 1)))
    else:
        for r in range(lv - 1):
            for c in range(lh):
                if (r + 2 * (c % 2)) % 4 == k:
                    out.append((qubit(lh, r, c), qubit(lh, r + 1, c)))
    return out


def generate(lv: int, lh: int, depth: int, seed: int) -> Circuit:
    """Random circuit of depth (1+depth+1) on an lv x lh lattice."""
    if lv < 1 or lh < 1 or depth < 0:
        raise ValueError("bad lattice or depth")
    rng = np.random.Generator(np.random.PCG64(seed))
    n = lv * lh
    gates: List[Gate] = [Gate(0, "H", q) for q in range(n)]
    last = [None] * n
    for t in range(1, depth + 1):
        pat = coupler_pattern(lv, lh, (t - 1) % 8)
        busy = set()
        for a, b in pat:
            gates.append(Gate(t, "CZ", a, b))
            busy.add(a)
            busy.add(b)
        for q in range(n):
            if q in busy:
                continue
            if last[q] is None:
                g = "T"
            else:
                options = [x for x in ONE_QUBIT_CHOICES if x != last[q]]
                g = options[int(rng.integers(0, 2))]
            last[q] = g
            gates.append(Gate(t, g, q))
    gates += [Gate(depth + 1, "H", q) for q in range(n)]
    return Circuit(lv, lh, depth, seed, gates)


def random_unitary(rng: np.random.Generator, dim: int) -> np.ndarray:
    """Haar-random unitary via QR of a complex Gaussian matrix (input data)."""
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))


def _flat(u: np.ndarray) -> List[float]:
    return [float(x) for v in u.reshape(-1) for x in (v.real, v.imag)]


def generate_general(lv: int, lh: int, layers: int, seed: int, two_qubit: str = "U2") -> Circuit:
    """Circuit of arbitrary 1q unitaries and nearest-neighbour 2q gates.

    Used to exercise the general-purpose path (any 1q gate, any 2q gate split by
    SVD, eq. (4)).  two_qubit is "U2" (Haar 4x4) or "CZ".
    """
    rng = np.random.Generator(np.random.PCG64([seed, 7]))
    n = lv * lh
    gates: List[Gate] = []
    for t in range(layers):
        for q in range(n):
            gates.append(Gate(2 * t, "U1", q, -1, _flat(random_unitary(rng, 2))))
        pat = coupler_pattern(lv, lh, t % 8)
        for a, b in pat:
            if two_qubit == "U2":
                gates.append(Gate(2 * t + 1, "U2", a, b, _flat(random_unitary(rng, 4))))
            else:
                gates.append(Gate(2 * t + 1, "CZ", a, b))
    return Circuit(lv, lh, layers, seed, gates, family="general-" + two_qubit)


def bitstrings(lv: int, lh: int, seed: int, count: int) -> np.ndarray:
    """Uniform random output bitstrings, shape (count, lv*lh), uint8."""
    rng = np.random.Generator(np.random.PCG64([seed, 1]))
    return rng.integers(0, 2, size=(count, lv * lh), dtype=np.uint8)


def all_bitstrings(n: int) -> np.ndarray:
    """Every bitstring of n qubits; row i has qubit 0 as its most significant bit."""
    idx = np.arange(2 ** n, dtype=np.int64)
    shifts = np.arange(n - 1, -1, -1, dtype=np.int64)
    return ((idx[:, None] >> shifts[None, :]) & 1).astype(np.uint8)


def last_row_variants(base: Sequence[int], lv: int, lh: int, cols: Sequence[int]) -> np.ndarray:
    """2**len(cols) bitstrings equal to `base` except on last-row columns `cols`.

    Variant i sets column cols[j] to bit j (most significant first) of i.  These
    bitstrings share every row but the last, so their amplitudes share the
    boundary tensor of the first lv-1 rows.
    """
    base = np.asarray(base, dtype=np.uint8)
    k = len(cols)
    out = np.repeat(base[None, :], 2 ** k, axis=0)
    for i in range(2 ** k):
        for j, c in enumerate(cols):
            out[i, qubit(lh, lv - 1, c)] = (i >> (k - 1 - j)) & 1
    return out
