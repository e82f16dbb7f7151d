"""Pins of the oracle's ||A||_inf (CPU only).

The norm sets every convergence threshold, rtol * ||A|| with the section-4
tolerance read as the infinity norm.  It is pinned here to hand-computed
largest absolute row sums of small nonsymmetric matrices whose row and column
sums differ, with empty first, interior and last rows, and a planted
column-sum mistake must fail the pin."""
import numpy as np

import oracle as O
from paper_1806_08020_amd import workloads as W


def _csr(n, rows):
    """CSR from {row: [(col, val), ...]} (rows missing from the dict are empty)."""
    rp = [0]
    ci, va = [], []
    for i in range(n):
        for c, v in sorted(rows.get(i, [])):
            ci.append(c)
            va.append(v)
        rp.append(len(ci))
    return W.CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va, np.float64))


# 5 x 5, rows 0, 2 and 4 empty:
#   row 1:  3 at col 1, -4 at col 2            |row sum| 7
#   row 3: -1 at col 0,  2 at col 3, -6 at col 4  |row sum| 9
# absolute column sums: 1, 3, 4, 2, 6 (largest 6, not 9)
HOLES = {1: [(1, 3.0), (2, -4.0)], 3: [(0, -1.0), (3, 2.0), (4, -6.0)]}


def test_empty_first_interior_last_rows():
    assert O.infnorm(_csr(5, HOLES)) == 9.0


def test_last_row_carries_the_maximum_after_an_empty_row():
    # row 2 empty, row 3 (the last) holds the largest sum: 0.5 + 7.25 = 7.75
    rows = {0: [(0, 1.0), (3, -2.0)], 1: [(2, 2.5)], 3: [(1, 0.5), (3, -7.25)]}
    assert O.infnorm(_csr(4, rows)) == 7.75


def test_single_entry_and_all_empty():
    assert O.infnorm(_csr(3, {2: [(0, -4.5)]})) == 4.5
    assert O.infnorm(_csr(3, {})) == 0.0
    assert O.infnorm(_csr(1, {0: [(0, -2.0)]})) == 2.0


def test_stencil_interior_row_sum():
    # the centred 2-D convection-diffusion stencil at beta*h = 0.5: interior
    # rows hold |4| + |-1 - 0.25| + |-1 + 0.25| + 1 + 1 = 8
    assert abs(O.infnorm(W.convdiff_2d(12, 0.5)) - 8.0) < 1e-15
    # 3-D, beta*h = 0.3 on every axis: 6 + 3 * (1.15 + 0.85) = 12
    assert abs(O.infnorm(W.convdiff_3d(6, 0.3)) - 12.0) < 1e-14   # 1.15 and 0.85 are inexact in binary


def _column_sum_norm(csr):
    # planted mistake: the largest absolute column sum (the 1-norm)
    a = np.abs(csr.vals)
    return float(np.bincount(csr.colind, weights=a, minlength=csr.n).max())


def test_planted_column_sum_mistake_is_caught():
    A = _csr(5, HOLES)
    assert _column_sum_norm(A) != 9.0
    assert _column_sum_norm(A) == 6.0
