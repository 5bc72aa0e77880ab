"""Closed-form complexity of the contraction schemes and exact step counts.

Closed forms (element counts for space, complex multiply-adds for time):
  eq. (8)            chi <= 2^ceil(d/8)
  eqs. (S7), (S8)    generic row scheme, L = min(Lv, Lh):
                     C^s = 2^(ceil(d/8) (L+1)),
                     C^t = (Lh-2)(Lv-2) 2^(ceil(d/8) (L+3))
  eqs. (S9), (S10)   even square:  C^s = 2^(ceil(d/8) sqrt(N) + 1),
                                   C^t = 2^(3 ceil(d/8) sqrt(N) / 2 + 1)
  eqs. (S11), (S12)  odd square:   C^s = 2^(ceil(d/8)(sqrt(N)+1)) + 2^(ceil(d/8) sqrt(N)),
                                   C^t = (2^ceil(d/8) + 1) 2^(ceil(d/8)(3 sqrt(N) - 1)/2)
  supplement S-III   Bristlecone-72 at depth (1+32+1): 2^(32/8 * 11 + 1) elements.
The paper quotes memory in bytes of complex128 elements (16 B each), which is
how its 32 TB / 0.5 PB / 16 PB / 8 PB / 16 TB figures come out.

`row_scheme_cmac` counts the exact work of absorbing sites one at a time
(each step costs |running tensor| * |site tensor| / |shared legs|), which is
what the generic scheme does; the leading term of that count is (S8).
"""
import math
from typing import Dict, Tuple

BYTES_C128 = 16


def chi_bound(d: int) -> int:
    return 2 ** math.ceil(d / 8)


def generic_space(lv: int, lh: int, d: int) -> int:
    L = min(lv, lh)
    return 2 ** (math.ceil(d / 8) * (L + 1))


def generic_time(lv: int, lh: int, d: int) -> int:
    L = min(lv, lh)
    return (lh - 2) * (lv - 2) * 2 ** (math.ceil(d / 8) * (L + 3))


def even_square_space(L: int, d: int) -> int:
    return 2 ** (math.ceil(d / 8) * L + 1)


def even_square_time(L: int, d: int) -> int:
    e = 3 * math.ceil(d / 8) * L
    assert e % 2 == 0
    return 2 ** (e // 2 + 1)


def odd_square_space(L: int, d: int) -> int:
    k = math.ceil(d / 8)
    return 2 ** (k * (L + 1)) + 2 ** (k * L)


def odd_square_time(L: int, d: int) -> int:
    k = math.ceil(d / 8)
    e = k * (3 * L - 1)
    assert e % 2 == 0
    return (2 ** k + 1) * 2 ** (e // 2)


def bristlecone_space(d: int = 32) -> int:
    return 2 ** (d // 8 * 11 + 1)


def row_scheme_cmac(lv: int, lh: int, dims: Dict[Tuple[str, int, int], int],
                    scheme: str = "rows") -> int:
    """Exact CMAC count of the site-by-site absorption in the given order."""
    from .peps import site_order

    def legs(r, c):
        out = {}
        if c > 0:
            out[("h", r, c - 1)] = dims[("h", r, c - 1)]
        if c + 1 < lh:
            out[("h", r, c)] = dims[("h", r, c)]
        if r > 0:
            out[("v", r - 1, c)] = dims[("v", r - 1, c)]
        if r + 1 < lv:
            out[("v", r, c)] = dims[("v", r, c)]
        return out

    acc = None
    total = 0
    for (r, c) in site_order(lv, lh, scheme):
        s = legs(r, c)
        if acc is None:
            acc = dict(s)
            continue
        shared = [k for k in s if k in acc]
        size_acc = math.prod(acc.values())
        size_new = math.prod(v for k, v in s.items() if k not in shared)
        total += size_acc * size_new
        for k in shared:
            del acc[k]
        for k, v in s.items():
            if k not in shared:
                acc[k] = v
    return total


def row_scheme_cmac_per_row(lv: int, lh: int, dims: Dict[Tuple[str, int, int], int]):
    """Exact CMAC of the row scheme (top-down, left to right) split by row."""
    out = []
    for r in range(lv):
        out.append(_count_prefix(lv, lh, dims, r + 1) - (_count_prefix(lv, lh, dims, r) if r else 0))
    return out


def _count_prefix(lv, lh, dims, n_rows):
    from .peps import site_order
    order = [p for p in site_order(lv, lh, "rows") if p[0] < n_rows]
    acc = None
    total = 0
    for (r, c) in order:
        s = {}
        if c > 0:
            s[("h", r, c - 1)] = dims[("h", r, c - 1)]
        if c + 1 < lh:
            s[("h", r, c)] = dims[("h", r, c)]
        if r > 0:
            s[("v", r - 1, c)] = dims[("v", r - 1, c)]
        if r + 1 < lv:
            s[("v", r, c)] = dims[("v", r, c)]
        if acc is None:
            acc = dict(s)
            continue
        shared = [k for k in s if k in acc]
        total += math.prod(acc.values()) * math.prod(v for k, v in s.items() if k not in shared)
        for k in shared:
            del acc[k]
        for k, v in s.items():
            if k not in shared:
                acc[k] = v
    return total


def uniform_dims(lv: int, lh: int, D: int) -> Dict[Tuple[str, int, int], int]:
    out = {}
    for r in range(lv):
        for c in range(lh):
            if c + 1 < lh:
                out[("h", r, c)] = D
            if r + 1 < lv:
                out[("v", r, c)] = D
    return out
