"""Invariants of the seeded random-circuit generator (supplement S-I rules)."""
import json
import os
from collections import Counter

import numpy as np
import pytest

import rqcgen


@pytest.mark.parametrize("lv,lh", [(3, 3), (4, 5), (5, 5), (6, 6), (7, 7), (2, 9)])
def test_patterns_are_matchings_and_partition_edges(lv, lh):
    edges = set(rqcgen.lattice_edges(lv, lh))
    seen = Counter()
    for p in range(8):
        pat = rqcgen.coupler_pattern(lv, lh, p)
        qubits = [q for e in pat for q in e]
        assert len(qubits) == len(set(qubits)), "pattern is not a matching"
        for e in pat:
            assert e in edges
            seen[e] += 1
    assert set(seen) == edges and all(v == 1 for v in seen.values())


@pytest.mark.parametrize("lv,lh,d", [(3, 3, 8), (4, 5, 24), (5, 5, 32), (6, 6, 40), (3, 4, 13)])
def test_cz_per_edge_and_counts(lv, lh, d):
    c = rqcgen.generate(lv, lh, d, 0)
    cz = Counter(tuple(sorted((g.q0, g.q1))) for g in c.gates if g.kind == "CZ")
    for e in rqcgen.lattice_edges(lv, lh):
        assert cz[tuple(sorted(e))] in (d // 8, -(-d // 8))
        if d % 8 == 0:
            assert cz[tuple(sorted(e))] == d // 8
    n = lv * lh
    n1q = sum(1 for g in c.gates if g.kind in ("T", "SX", "SY"))
    assert n1q == d * n - 2 * sum(cz.values())
    assert sum(1 for g in c.gates if g.kind == "H") == 2 * n


def test_one_qubit_rules():
    c = rqcgen.generate(5, 5, 32, 3)
    per_q = {}
    for g in c.gates:
        if g.kind in ("T", "SX", "SY"):
            per_q.setdefault(g.q0, []).append(g.kind)
    for q, seq in per_q.items():
        assert seq[0] == "T"
        assert all(a != b for a, b in zip(seq, seq[1:]))
    # within a cycle, gates act on disjoint qubits and CZ qubits get no 1q gate
    by_cycle = {}
    for g in c.gates:
        by_cycle.setdefault(g.cycle, []).append(g)
    for t, gs in by_cycle.items():
        qs = [q for g in gs for q in ((g.q0, g.q1) if g.kind == "CZ" else (g.q0,))]
        assert len(qs) == len(set(qs))
        if 1 <= t <= 32:
            assert len(qs) == 25


def test_deterministic_and_serialisable():
    a = rqcgen.generate(4, 5, 24, 7)
    b = rqcgen.generate(4, 5, 24, 7)
    assert a.sha256() == b.sha256()
    assert rqcgen.generate(4, 5, 24, 8).sha256() != a.sha256()
    c = rqcgen.Circuit.from_json(a.to_json())
    assert c.sha256() == a.sha256()
    g = rqcgen.generate_general(2, 3, 3, 1)
    assert rqcgen.Circuit.from_json(g.to_json()).sha256() == g.sha256()


def test_golden_hashes(golden_dir):
    with open(os.path.join(golden_dir, "circuits.json")) as f:
        gold = json.load(f)
    for key, h in gold.items():
        lv, lh, d, seed = (int(x) for x in key.split("_"))
        assert rqcgen.generate(lv, lh, d, seed).sha256() == h, key


def test_bitstrings_and_variants():
    b = rqcgen.bitstrings(6, 6, 0, 4)
    assert b.shape == (4, 36) and b.dtype == np.uint8 and set(np.unique(b)) <= {0, 1}
    assert np.array_equal(b, rqcgen.bitstrings(6, 6, 0, 4))
    v = rqcgen.last_row_variants(b[0], 6, 6, [2, 3, 4, 5])
    assert v.shape == (16, 36)
    assert len({row.tobytes() for row in v}) == 16
    assert np.all(v[:, :30] == b[0][:30])
    assert any(np.array_equal(row, b[0]) for row in v)
    allb = rqcgen.all_bitstrings(3)
    assert allb.tolist()[1] == [0, 0, 1] and allb.tolist()[4] == [1, 0, 0]
