"""Closed forms against the numbers the paper prints, and the exact step count
of the row scheme against its leading term (S8)."""
import json
import os

import pytest

import rqcgen
from oracle import complexity as cx
from oracle import peps


def _golden(golden_dir):
    with open(os.path.join(golden_dir, "paper_numbers.json")) as f:
        return json.load(f)


def test_paper_memory_numbers(golden_dir):
    g = _golden(golden_dir)["memory_bytes_c128"]
    TiB, PiB = 2 ** 40, 2 ** 50
    B = cx.BYTES_C128
    # main text: 8x8 (1+40+1) 32 TB, same as 10x10 (1+32+1)
    assert cx.even_square_space(8, 40) * B == g["8x8_d40"] == 32 * TiB
    assert cx.even_square_space(10, 32) == cx.even_square_space(8, 40)
    # 8 x l, l > 8 (generic scheme, L = 8): about 0.5 PB
    assert cx.generic_space(8, 12, 40) * B == g["8xl_d40"] == PiB // 2
    # 9x9 (1+40+1): 16 PB (odd partition; the leading term is 2^50 elements)
    assert abs(cx.odd_square_space(9, 40) * B / g["9x9_d40"] - 1) < 0.04
    # 12x12 (1+32+1): 8 PB
    assert cx.even_square_space(12, 32) * B == g["12x12_d32"] == 8 * PiB
    # 7x7 (1+40+1): theoretical 16 TB (supplement S-IV)
    assert cx.generic_space(7, 7, 40) * B == g["7x7_d40"] == 16 * TiB
    # Bristlecone-72 at (1+32+1): 2^45 elements, below 0.6 PB
    assert cx.bristlecone_space(32) == 2 ** 45
    assert cx.bristlecone_space(32) * B < 0.6e15 * 1.2


@pytest.mark.parametrize("lv,lh,d,ratio", [(6, 6, 40, 1.0159), (5, 5, 32, 1.0435), (3, 3, 8, 3.0625)])
def test_exact_count_vs_S8(lv, lh, d, ratio):
    D = cx.chi_bound(d)
    exact = cx.row_scheme_cmac(lv, lh, cx.uniform_dims(lv, lh, D))
    assert abs(exact / cx.generic_time(lv, lh, d) - ratio) < 5e-4


def test_exact_count_matches_built_peps():
    c = rqcgen.generate(4, 5, 24, 0)
    P = peps.build(c)
    dims = peps.bond_dims(P)
    assert cx.row_scheme_cmac(4, 5, dims, "cols") == cx.row_scheme_cmac(4, 5, cx.uniform_dims(4, 5, 8), "cols")
    # sweeping along the short side is cheaper (largest tensor rank min(Lv,Lh)+1)
    assert cx.row_scheme_cmac(4, 5, dims, "cols") < cx.row_scheme_cmac(4, 5, dims, "rows")


def test_leading_term_6x6():
    # interior row of 6x6 D=32: 4 sites of M = D^5, K = N = D^2 -> 4 * 2^45
    assert cx.generic_time(6, 6, 40) == 16 * 2 ** 45
    assert cx.generic_space(6, 6, 40) == 2 ** 35


def _closed_form_rows(L, D, lv):
    """Per-row multiply-adds of the row scheme on an Lv x L lattice with every
    bond D, written out from the shapes of eqs. S2-S6 (site by site, left to
    right): first row D^(c+3) for sites c = 1..L-2 plus D^(L+1) at the last
    site; an interior row 2 D^(L+2) + (L-2) D^(L+3); the last row D^(L+1) +
    sum_{c=1}^{L-2} D^(L-c+2) + D^2."""
    first = sum(D ** (c + 3) for c in range(1, L - 1)) + D ** (L + 1)
    inner = 2 * D ** (L + 2) + (L - 2) * D ** (L + 3)
    last = D ** (L + 1) + sum(D ** (L - c + 2) for c in range(1, L - 1)) + D ** 2
    return [first] + [inner] * (lv - 2) + [last]


@pytest.mark.parametrize("lv,L,D", [(3, 3, 2), (5, 5, 16), (6, 6, 32), (7, 7, 32), (5, 4, 8), (4, 6, 4)])
def test_per_row_counts_closed_form(lv, L, D):
    """The per-row split the bench extrapolates with equals the closed form of
    each row, and the rows add up to the whole-scheme count."""
    dims = cx.uniform_dims(lv, L, D)
    per_row = cx.row_scheme_cmac_per_row(lv, L, dims)
    assert per_row == _closed_form_rows(L, D, lv)
    assert sum(per_row) == cx.row_scheme_cmac(lv, L, dims)


@pytest.mark.parametrize("lv,lh,d,seed", [(8, 8, 25, 0), (4, 5, 13, 1), (3, 6, 21, 2), (6, 6, 17, 3)])
def test_per_row_counts_sum_with_uneven_bonds(lv, lh, d, seed):
    """Uneven bonds (d not a multiple of 8): the per-row counts of a built
    PEPS add up to the total, and the first and last rows are the cheapest."""
    P = peps.build(rqcgen.generate(lv, lh, d, seed))
    dims = peps.bond_dims(P)
    assert len(set(dims.values())) > 1
    per_row = cx.row_scheme_cmac_per_row(lv, lh, dims)
    assert len(per_row) == lv and all(x > 0 for x in per_row)
    assert sum(per_row) == cx.row_scheme_cmac(lv, lh, dims)
    if lv > 2:
        assert per_row[0] <= max(per_row[1:-1]) and per_row[-1] <= max(per_row[1:-1])
