"""O3: PEPS evolution and exact overlap contraction on the CPU, in FP64.

Evolution (main text, "Quantum Circuit Simulator Based on PEPS"):
  * the state is a product of rank-5 site tensors A_n[sigma, l, r, u, d]
    (eq. 1), initialised to |0> with all bonds of size 1;
  * a one-qubit gate contracts the physical index (eq. 3);
  * a two-qubit gate O on a nearest-neighbour pair is factorised by SVD as
    sum_s U_s (x) V_s with the singular values absorbed (eq. 4; here split
    as sqrt(S) on both sides, which leaves the product unchanged), and the
    new index s is bundled with the shared bond on both sites (eqs. 5-6).
    The paper writes r' = (r, s) and l' = (s, l); any consistent pair is
    correct, and we use (old, new) on both sides: new = old * chi_o + s.
Overlap: E_n = A_n[tau_n] (eq. 7), and <tau|psi> is the contraction of the
network of E_n.

Contractions work on labelled tensors: every leg carries the identity of its
bond, ('h', r, c) for the bond between (r, c) and (r, c+1) and ('v', r, c)
for the bond between (r, c) and (r+1, c).  Contracting two labelled tensors
sums over the labels they share (a plain numpy tensordot), so a contraction
order is just an order of sites:
  * row scheme (supplement S-II, eqs. S2-S6): absorb sites row by row, left
    to right; after row i the running tensor is F_i with the down legs of
    row i open; the last step leaves the scalar amplitude;
  * square partition for even L x L lattices (eqs. S9-S10): contract each
    quadrant, then the upper pair, the lower pair, and the two results;
  * loop slicing (the "cut" technique named in the conclusions): fixing a
    bond to one value and summing the sliced results over that value.
"""
from __future__ import annotations

from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

from . import gates as G

Label = Tuple[str, int, int]


# --------------------------------------------------------------------------
# evolution, eqs. (3)-(6)
# --------------------------------------------------------------------------

class PEPS:
    def __init__(self, lv: int, lh: int):
        self.lv, self.lh = lv, lh
        self.A: List[np.ndarray] = []
        for _ in range(lv * lh):
            a = np.zeros((2, 1, 1, 1, 1), dtype=np.complex128)
            a[0, 0, 0, 0, 0] = 1.0
            self.A.append(a)

    def pos(self, q: int) -> Tuple[int, int]:
        return divmod(q, self.lh)

    def chi(self) -> int:
        """Bond dimension, eq. (2): the largest auxiliary dimension."""
        return max(max(a.shape[1:]) for a in self.A)


def svd_split(o: np.ndarray, tol: float = 1e-12):
    """Eq. (4): O[(tn tm), (sn sm)] = sum_s U[tn, sn, s] V[s, tm, sm]."""
    o4 = o.reshape(2, 2, 2, 2)                     # [tn, tm, sn, sm]
    m = o4.transpose(0, 2, 1, 3).reshape(4, 4)     # rows (tn sn), cols (tm sm)
    u, s, vh = np.linalg.svd(m)
    k = int(np.sum(s > tol * s[0]))
    root = np.sqrt(s[:k])
    un = (u[:, :k] * root[None, :]).reshape(2, 2, k)
    vm = (root[:, None] * vh[:k, :]).reshape(k, 2, 2)
    return un, vm


def apply_1q(peps: PEPS, u: np.ndarray, q: int) -> None:
    peps.A[q] = np.einsum("ts,slrud->tlrud", u, peps.A[q])


def apply_2q(peps: PEPS, o: np.ndarray, q0: int, q1: int) -> None:
    (r0, c0), (r1, c1) = peps.pos(q0), peps.pos(q1)
    if (r0, c0 + 1) == (r1, c1) or (r0 + 1, c0) == (r1, c1):
        n, m, op = q0, q1, o
    elif (r1, c1 + 1) == (r0, c0) or (r1 + 1, c1) == (r0, c0):
        # put the left/upper qubit first: swap both the output and input pairs
        n, m = q1, q0
        op = o.reshape(2, 2, 2, 2).transpose(1, 0, 3, 2).reshape(4, 4)
    else:
        raise ValueError(f"two-qubit gate on non-neighbouring qubits {q0}, {q1}")
    un, vm = svd_split(op)
    k = un.shape[2]
    a, b = peps.A[n], peps.A[m]
    _, l, r, u, d = a.shape
    _, l2, r2, u2, d2 = b.shape
    if peps.pos(m)[0] == peps.pos(n)[0]:  # horizontal: n.r <-> m.l
        na = np.einsum("tsk,slrud->tlrkud", un, a).reshape(2, l, r * k, u, d)
        nb = np.einsum("kts,slrud->tlkrud", vm, b).reshape(2, l2 * k, r2, u2, d2)
    else:                                   # vertical: n.d <-> m.u
        na = np.einsum("tsk,slrud->tlrudk", un, a).reshape(2, l, r, u, d * k)
        nb = np.einsum("kts,slrud->tlrukd", vm, b).reshape(2, l2, r2, u2 * k, d2)
    peps.A[n], peps.A[m] = na, nb


def build(circuit) -> PEPS:
    """Absorb every gate of the circuit, in order, into the site tensors."""
    peps = PEPS(circuit.lv, circuit.lh)
    for g in circuit.gates:
        mat = G.matrix_of(g)
        if G.is_two_qubit(g):
            apply_2q(peps, mat, g.q0, g.q1)
        else:
            apply_1q(peps, mat, g.q0)
    return peps


def bond_dims(peps: PEPS) -> Dict[Label, int]:
    out = {}
    for q, a in enumerate(peps.A):
        r, c = peps.pos(q)
        if c + 1 < peps.lh:
            out[("h", r, c)] = a.shape[2]
        if r + 1 < peps.lv:
            out[("v", r, c)] = a.shape[4]
    return out


# --------------------------------------------------------------------------
# labelled tensors
# --------------------------------------------------------------------------

class LT:
    """A tensor with one bond label per axis."""

    __slots__ = ("a", "labels")

    def __init__(self, a: np.ndarray, labels: Sequence[Label]):
        assert a.ndim == len(labels)
        self.a, self.labels = a, list(labels)

    def dim(self, label: Label) -> int:
        return self.a.shape[self.labels.index(label)]

    def ordered(self, labels: Sequence[Label]) -> np.ndarray:
        return np.transpose(self.a, [self.labels.index(x) for x in labels])


def contract(x: LT, y: LT) -> LT:
    """Sum over every label the two tensors share."""
    shared = [l for l in x.labels if l in y.labels]
    ax = [x.labels.index(l) for l in shared]
    ay = [y.labels.index(l) for l in shared]
    out = np.tensordot(x.a, y.a, axes=(ax, ay))
    labels = [l for l in x.labels if l not in shared] + [l for l in y.labels if l not in shared]
    return LT(out, labels)


def fix(t: LT, label: Label, value: int) -> LT:
    """Slice one bond at a fixed value (one term of a cut loop)."""
    if label not in t.labels:
        return t
    i = t.labels.index(label)
    return LT(np.take(t.a, value, axis=i), t.labels[:i] + t.labels[i + 1:])


def projected_sites(peps: PEPS, bits: Sequence[int]) -> Dict[Tuple[int, int], LT]:
    """E_n = A_n[tau_n] as labelled rank-<=4 tensors (eq. 7)."""
    out = {}
    for q, a in enumerate(peps.A):
        r, c = peps.pos(q)
        e = a[int(bits[q])]
        legs = [("h", r, c - 1), ("h", r, c), ("v", r - 1, c), ("v", r, c)]
        inside = [c > 0, c + 1 < peps.lh, r > 0, r + 1 < peps.lv]
        keep_axes, labels = [], []
        for ax, (lab, ok) in enumerate(zip(legs, inside)):
            if ok:
                keep_axes.append(ax)
                labels.append(lab)
            elif e.shape[ax] != 1:
                raise ValueError("boundary leg with dimension > 1")
        e = e.reshape([e.shape[ax] for ax in keep_axes])
        out[(r, c)] = LT(e, labels)
    return out


def contract_sites(sites: Dict[Tuple[int, int], LT], order: Iterable[Tuple[int, int]],
                   start: Optional[LT] = None, fixed: Optional[Dict[Label, int]] = None) -> LT:
    """Absorb sites one at a time in the given order; `fixed` slices bonds."""
    fixed = fixed or {}
    acc = start
    if acc is not None:
        for lab, v in fixed.items():
            acc = fix(acc, lab, v)
    for p in order:
        t = sites[p]
        for lab, v in fixed.items():
            t = fix(t, lab, v)
        acc = t if acc is None else contract(acc, t)
    return acc


# --------------------------------------------------------------------------
# contraction orders
# --------------------------------------------------------------------------

def site_order(lv: int, lh: int, scheme: str) -> List[Tuple[int, int]]:
    """Site orders of the generic scheme (Fig. S2(a)) and its mirror images."""
    if scheme == "rows":        # top-down, left to right (eqs. S2-S6)
        return [(r, c) for r in range(lv) for c in range(lh)]
    if scheme == "rows_rl":     # top-down, right to left
        return [(r, c) for r in range(lv) for c in reversed(range(lh))]
    if scheme == "rows_bu":     # bottom-up, left to right
        return [(r, c) for r in reversed(range(lv)) for c in range(lh)]
    if scheme == "cols":        # left to right by columns (used when Lh > Lv)
        return [(r, c) for c in range(lh) for r in range(lv)]
    raise ValueError(scheme)


def amplitude(peps: PEPS, bits: Sequence[int], scheme: str = "rows") -> complex:
    """<tau|psi> by absorbing sites in the order of `scheme`."""
    sites = projected_sites(peps, bits)
    if scheme == "quadrants":
        return amplitude_quadrants(peps, bits)
    res = contract_sites(sites, site_order(peps.lv, peps.lh, scheme))
    assert res.a.ndim == 0
    return complex(res.a)


def amplitudes(peps: PEPS, bits: np.ndarray, scheme: str = "rows") -> np.ndarray:
    return np.array([amplitude(peps, b, scheme) for b in np.asarray(bits)], dtype=np.complex128)


def boundary_after_rows(peps: PEPS, bits: Sequence[int], n_rows: int) -> LT:
    """F_{n_rows}: the first n_rows rows contracted, down legs of the last open (S2-S5)."""
    sites = projected_sites(peps, bits)
    return contract_sites(sites, [(r, c) for r in range(n_rows) for c in range(peps.lh)])


def row_transfer(F: LT, sites: Dict[Tuple[int, int], LT], row: int, lh: int,
                 fixed: Optional[Dict[Label, int]] = None) -> LT:
    """One row of the generic scheme: G_1 (S3), G_j (S4), F_row = G_Lh (S5)."""
    return contract_sites(sites, [(row, c) for c in range(lh)], start=F, fixed=fixed)


# --------------------------------------------------------------------------
# square partition, eqs. (S9)-(S10)
# --------------------------------------------------------------------------

def quadrant_sites(L: int, which: str) -> List[Tuple[int, int]]:
    """Sites of one m x m quadrant (m = L/2), in the order they are absorbed.

    Each quadrant is swept from its outer corner toward the centre of the
    lattice (upper quadrants top-down, lower ones bottom-up; left quadrants
    left to right, right ones right to left), so that the bonds it leaves open
    toward its neighbours are created late and intermediates stay small.
    """
    m = L // 2
    rows = list(range(0, m)) if which[0] == "u" else list(reversed(range(m, L)))
    cols = list(range(0, m)) if which[1] == "l" else list(reversed(range(m, L)))
    return [(r, c) for r in rows for c in cols]


def amplitude_quadrants(peps: PEPS, bits: Sequence[int]) -> complex:
    """Even square lattice: four m x m quadrants, then (ul.ur).(bl.br)."""
    L = peps.lv
    if peps.lh != L or L % 2:
        raise ValueError("the quadrant partition needs an even square lattice")
    sites = projected_sites(peps, bits)
    q = {w: contract_sites(sites, quadrant_sites(L, w)) for w in ("ul", "ur", "bl", "br")}
    top = contract(q["ul"], q["ur"])
    bottom = contract(q["bl"], q["br"])
    res = contract(top, bottom)
    assert res.a.ndim == 0
    return complex(res.a)


def quadrant_amplitudes_sliced(peps: PEPS, base_bits: Sequence[int], left_patterns: np.ndarray,
                               right_patterns: np.ndarray, log=None) -> np.ndarray:
    """Square-partition amplitudes of many bitstrings with bounded memory.

    The bitstrings differ only in the bottom-left quadrant (rows of
    `left_patterns`, full bitstrings) and the bottom-right quadrant
    (`right_patterns`); result[i, j] is the amplitude of the bitstring that
    takes its bottom-left bits from left_patterns[i], its bottom-right bits
    from right_patterns[j] and all other bits from base_bits.

    With e, a, b, c the bond groups ul|ur, ul|bl, ur|br, bl|br:
        amp = sum ul[e,a] ur[e,b] bl[a,c] br[b,c]
            = sum_z sum_{b,c'} X_z[b,c'] br_z[b,c'],   X_z = T^T bl_z,
        T^T[b,a] = sum_x ur_x[e',b]^T ul_x[e',a],
    where x runs over the top bond of group e and z over the bottom bond of
    group c (cut loops).  Only T^T and slices of the other tensors are held.
    """
    L = peps.lv
    m = L // 2
    if peps.lh != L or L % 2:
        raise ValueError("needs an even square lattice")
    e_lab = [("h", r, m - 1) for r in range(m)]
    a_lab = [("v", m - 1, c) for c in range(m)]
    b_lab = [("v", m - 1, c) for c in range(m, L)]
    c_lab = [("h", r, m - 1) for r in range(m, L)]
    dims = bond_dims(peps)
    de = int(np.prod([dims[x] for x in e_lab]))
    da = int(np.prod([dims[x] for x in a_lab]))
    db = int(np.prod([dims[x] for x in b_lab]))
    dc = int(np.prod([dims[x] for x in c_lab]))
    say = log or (lambda *_: None)

    base_sites = projected_sites(peps, base_bits)

    # T^T[b, a] = sum over slices x of e_0: ur_x[e', b]^T ul_x[e', a]
    tt = np.zeros((db, da), dtype=np.complex128)
    e0 = e_lab[0]
    for x in range(dims[e0]):
        ul = contract_sites(base_sites, quadrant_sites(L, "ul"), fixed={e0: x})
        ur = contract_sites(base_sites, quadrant_sites(L, "ur"), fixed={e0: x})
        ulm = ul.ordered(e_lab[1:] + a_lab).reshape(de // dims[e0], da)
        urm = ur.ordered(e_lab[1:] + b_lab).reshape(de // dims[e0], db)
        _accumulate_matmul(tt, urm.T, ulm)
        del ul, ur, ulm, urm
        say(f"T slice {x + 1}/{dims[e0]}")

    out = np.zeros((len(left_patterns), len(right_patterns)), dtype=np.complex128)
    zl = c_lab[-1]
    lsites = [projected_sites(peps, lp) for lp in left_patterns]
    rsites = [projected_sites(peps, rp) for rp in right_patterns]
    for z in range(dims[zl]):
        brs = []
        for rs in rsites:
            br = contract_sites(rs, quadrant_sites(L, "br"), fixed={zl: z})
            brs.append(br.ordered(b_lab + c_lab[:-1]).reshape(db, dc // dims[zl]))
        for i, ls in enumerate(lsites):
            bl = contract_sites(ls, quadrant_sites(L, "bl"), fixed={zl: z})
            blm = bl.ordered(a_lab + c_lab[:-1]).reshape(da, dc // dims[zl])
            xz = tt @ blm                                   # X[b, c'] at c_last = z
            for j, brm in enumerate(brs):
                out[i, j] += np.sum(xz * brm)
            del bl, blm, xz
        del brs
        say(f"bottom slice {z + 1}/{dims[zl]}")
    return out


def _accumulate_matmul(c: np.ndarray, a: np.ndarray, b: np.ndarray, rows: int = 4096) -> None:
    """c += a @ b, a block of rows at a time to bound the temporary."""
    for s in range(0, c.shape[0], rows):
        c[s:s + rows] += a[s:s + rows] @ b


# --------------------------------------------------------------------------
# row scheme with cut loops, for lattices whose boundary is too large to hold
# twice with every leg open (supplement S-II, eqs. S2-S6)
# --------------------------------------------------------------------------

def row_amplitudes_sliced(peps: PEPS, base_bits: Sequence[int], variants: np.ndarray, log=None) -> np.ndarray:
    """Row-scheme amplitudes of bitstrings that differ only in the last row.

    Rows 0..Lv-2 are contracted once with the bits of `base_bits`; the last
    row once per row of `variants` (full bitstrings; their other rows must
    equal the base).  Every row transfer is split by two cut loops: v, the
    down leg of the previous row at the last column (the leg the last site of
    the row absorbs), and w, the new down leg at column 0 (the leg the first
    site creates).  F_out[w] = sum_v row_transfer(F_in at v, w); each term
    holds tensors of D^(L-1) elements instead of D^(L+1).
    """
    lv, lh = peps.lv, peps.lh
    say = log or (lambda *_: None)
    variants = np.asarray(variants)
    for b in variants:
        if not np.array_equal(np.asarray(b)[: (lv - 1) * lh], np.asarray(base_bits)[: (lv - 1) * lh]):
            raise ValueError("variants must share rows 0..Lv-2 with the base")
    dims = bond_dims(peps)
    sites = projected_sites(peps, base_bits)

    def down(r):
        return [("v", r, c) for c in range(lh)]

    # row 0, one cut loop over its first down leg
    w0 = ("v", 0, 0)
    F = np.zeros([dims[x] for x in down(0)], dtype=np.complex128)
    for w in range(dims[w0]):
        part = contract_sites(sites, [(0, c) for c in range(lh)], fixed={w0: w})
        F[w] = part.ordered(down(0)[1:])
    say("row 0")
    for r in range(1, lv - 1):
        v_lab, w_lab = ("v", r - 1, lh - 1), ("v", r, 0)
        Fin = LT(F, down(r - 1))
        F = np.zeros([dims[x] for x in down(r)], dtype=np.complex128)
        for w in range(dims[w_lab]):
            for v in range(dims[v_lab]):
                part = row_transfer(fix(Fin, v_lab, v), sites, r, lh, fixed={v_lab: v, w_lab: w})
                F[w] += part.ordered(down(r)[1:])
            say(f"row {r}: w {w + 1}/{dims[w_lab]}")
        del Fin
    # last row: one cut loop over v for every variant
    Fin = LT(F, down(lv - 2))
    v_lab = ("v", lv - 2, lh - 1)
    out = np.zeros(len(variants), dtype=np.complex128)
    for i, b in enumerate(variants):
        s = projected_sites(peps, b)
        for v in range(dims[v_lab]):
            res = row_transfer(fix(Fin, v_lab, v), s, lv - 1, lh, fixed={v_lab: v})
            out[i] += complex(res.a)
    say("last row")
    return out


def halves_amplitude_sliced(peps: PEPS, bits: Sequence[int], log=None) -> complex:
    """One amplitude of an even L x L lattice by the square partition grouped
    into left and right halves (the four blocks of eqs. S9-S10 paired the
    other way): with e, a, b, c the bond groups ul|ur, ul|bl, ur|br, bl|br,
        amp = sum_{e,c} Lft[e,c] Rgt[e,c],  Lft = ul . bl (over a),  Rgt = ur . br (over b),
    cut over the first bond x of e and the last bond z of c, so each term
    holds D^(L-1)-element slices:
        amp = sum_{x,z} sum_{e',c'} (ul_x bl_z)[e',c'] (ur_x br_z)[e',c'].
    The lower quadrants' slices are kept, the upper ones made once per x."""
    L = peps.lv
    m = L // 2
    if peps.lh != L or L % 2:
        raise ValueError("needs an even square lattice")
    e_lab = [("h", r, m - 1) for r in range(m)]
    a_lab = [("v", m - 1, c) for c in range(m)]
    b_lab = [("v", m - 1, c) for c in range(m, L)]
    c_lab = [("h", r, m - 1) for r in range(m, L)]
    dims = bond_dims(peps)
    de = int(np.prod([dims[x] for x in e_lab]))
    da = int(np.prod([dims[x] for x in a_lab]))
    db = int(np.prod([dims[x] for x in b_lab]))
    dc = int(np.prod([dims[x] for x in c_lab]))
    say = log or (lambda *_: None)
    sites = projected_sites(peps, bits)
    x_lab, z_lab = e_lab[0], c_lab[-1]
    bl, br = [], []
    for z in range(dims[z_lab]):
        bl.append(contract_sites(sites, quadrant_sites(L, "bl"), fixed={z_lab: z})
                  .ordered(a_lab + c_lab[:-1]).reshape(da, dc // dims[z_lab]))
        br.append(contract_sites(sites, quadrant_sites(L, "br"), fixed={z_lab: z})
                  .ordered(b_lab + c_lab[:-1]).reshape(db, dc // dims[z_lab]))
    say("lower quadrant slices")
    amp = 0j
    for x in range(dims[x_lab]):
        ul = contract_sites(sites, quadrant_sites(L, "ul"), fixed={x_lab: x}) \
            .ordered(e_lab[1:] + a_lab).reshape(de // dims[x_lab], da)
        ur = contract_sites(sites, quadrant_sites(L, "ur"), fixed={x_lab: x}) \
            .ordered(e_lab[1:] + b_lab).reshape(de // dims[x_lab], db)
        for z in range(dims[z_lab]):
            amp += np.sum((ul @ bl[z]) * (ur @ br[z]))
        del ul, ur
        say(f"x {x + 1}/{dims[x_lab]}")
    return complex(amp)
