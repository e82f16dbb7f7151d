"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This module only *builds inputs*: sparse matrices in CSR form (int32 row
pointers, int32 sorted column indices, float64 values) and seeded start
vectors.  It holds none of the eigen-solver's arithmetic, so both sides of a
parity test can use it without sharing any part of the method.

Matrices follow the finite-difference operators used in the paper's
experiments (section 4, Example 1: second-order centred differences on the
unit square with homogeneous Dirichlet boundaries) and the synthetic shapes of
the measured workloads:

* ``laplacian_2d``          5-point Laplacian, stencil [4; -1 x 4]
* ``convdiff_2d``           -u_xx - u_yy + beta u_x, centred, scaled by h^2
* ``convdiff_3d``           -Lap u + beta (u_x + u_y + u_z), 7-point, scaled by h^2
* ``two_region_convdiff``   the two-region operator of Example 1
* ``random_banded``         random nonsymmetric band matrix (27 nnz per row)
* ``diag_csr``              diagonal matrices of Examples 4, 6, 7

Grid ordering is lexicographic with x fastest.  Every operator is scaled by h^2
(unscaled stencil), which changes eigenvalues by a constant factor only.

Seeds: a workload with integer seed ``s`` draws its matrix from
``numpy.random.default_rng([s, 0])`` and its vectors from
``numpy.random.default_rng([s, 1])`` (first draw b, the GMRES start vector;
second draw v0, the Arnoldi start vector: the paper uses two different random
vectors, section 4).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR", "laplacian_2d", "convdiff_2d", "convdiff_3d", "two_region_convdiff",
    "random_banded", "diag_csr", "dense_csr", "start_vectors", "stencil_nnz",
]


@dataclass
class CSR:
    """A square sparse matrix in CSR form (host arrays)."""
    n: int
    rowptr: np.ndarray   # int32, n+1
    colind: np.ndarray   # int32, nnz, sorted within each row
    vals: np.ndarray     # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.vals, self.colind, self.rowptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        return self.to_scipy().toarray()


def _from_coo(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CSR:
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32 indices")
    return CSR(n, rowptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64))


def _stencil(dims, center, lower, upper) -> CSR:
    """Generic constant-coefficient stencil on a tensor grid, Dirichlet.

    dims   : grid sizes (x fastest)
    center : diagonal coefficient
    lower  : coefficient of the -1 neighbour along each axis (tuple per axis)
    upper  : coefficient of the +1 neighbour along each axis

    Rows are built in place: the neighbour offsets, sorted, give each row's
    columns in increasing order, so no global sort is needed.
    """
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64)
    strides = np.cumprod((1,) + dims[:-1])
    # (offset, coefficient, validity mask) for every neighbour, offsets ascending
    entries = []
    rem = idx
    coords = []
    for d in dims:
        coords.append(rem % d)
        rem = rem // d
    for ax in reversed(range(len(dims))):
        entries.append((-int(strides[ax]), lower[ax], coords[ax] > 0))
    entries.append((0, center, np.ones(n, dtype=bool)))
    for ax in range(len(dims)):
        entries.append((int(strides[ax]), upper[ax], coords[ax] < dims[ax] - 1))
    mask = np.stack([e[2] for e in entries], axis=1)                 # n x s
    offs = np.array([e[0] for e in entries], dtype=np.int64)
    coef = np.array([e[1] for e in entries], dtype=np.float64)
    cols = (idx[:, None] + offs[None, :])[mask]
    vals = np.broadcast_to(coef, mask.shape)[mask]
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32 indices")
    return CSR(n, rowptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64))


def laplacian_2d(nx: int, ny: int | None = None) -> CSR:
    """5-point Laplacian on an nx-by-ny interior grid, h^2-scaled."""
    ny = nx if ny is None else ny
    return _stencil((nx, ny), 4.0, (-1.0, -1.0), (-1.0, -1.0))


def convdiff_2d(N: int, beta_h: float, M: int | None = None) -> CSR:
    """-u_xx - u_yy + beta u_x, centred differences, h^2-scaled.

    West / east couplings are -1 - beta*h/2 and -1 + beta*h/2.
    """
    M = N if M is None else M
    b = 0.5 * beta_h
    return _stencil((N, M), 4.0, (-1.0 - b, -1.0), (-1.0 + b, -1.0))


def convdiff_3d(N: int, beta_h: float) -> CSR:
    """-Lap u + beta (u_x + u_y + u_z), 7-point centred, h^2-scaled."""
    b = 0.5 * beta_h
    return _stencil((N, N, N), 6.0, (-1.0 - b,) * 3, (-1.0 + b,) * 3)


def two_region_convdiff(N: int) -> CSR:
    """Example 1 of section 4: -u_xx-u_yy+20u_x on the bottom half of the
    unit square, -100u_xx-100u_yy+2000u_x on the top half; h = 1/(N+1);
    h^2-scaled.  Rows whose y-coordinate lies above 1/2 use the top-half
    coefficients."""
    h = 1.0 / (N + 1)
    n = N * N
    idx = np.arange(n, dtype=np.int64)
    ix = idx % N
    iy = idx // N
    y = (iy + 1) * h
    top = y > 0.5
    diff = np.where(top, 100.0, 1.0)
    beta = np.where(top, 2000.0, 20.0)
    rows = [idx]; cols = [idx]; vals = [4.0 * diff]
    m = ix > 0
    rows.append(idx[m]); cols.append(idx[m] - 1); vals.append((-diff - 0.5 * beta * h)[m])
    m = ix < N - 1
    rows.append(idx[m]); cols.append(idx[m] + 1); vals.append((-diff + 0.5 * beta * h)[m])
    m = iy > 0
    rows.append(idx[m]); cols.append(idx[m] - N); vals.append((-diff)[m])
    m = iy < N - 1
    rows.append(idx[m]); cols.append(idx[m] + N); vals.append((-diff)[m])
    return _from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def random_banded(n: int, nnz_per_row: int = 27, band: int = 5000, seed: int = 4,
                  diag_max: float = 10.0) -> CSR:
    """Random nonsymmetric band matrix.

    Each row i holds a diagonal entry uniform on [0, diag_max] and
    ``nnz_per_row - 1`` distinct off-diagonal columns i+o with offsets o
    uniform on [-band, band] minus {0}; an offset that leaves the matrix or
    repeats another in its row is redrawn on its own.
    Off-diagonal values are N(0,1)/sqrt(nnz_per_row).  Columns sorted per row.
    """
    rng = np.random.default_rng([seed, 0])
    k = nnz_per_row - 1
    if n < 2 * band + 1 and n - 1 < k:
        raise ValueError("matrix too small for the requested row length")
    rows_idx = np.arange(n, dtype=np.int64)
    span = 2 * band

    def draw(size):
        o = rng.integers(1, span + 1, size=size)                  # 1..2*band
        return np.where(o > band, o - span - 1, o)                # -> [-band,-1] u [1,band]

    offs = draw((n, k))
    active = rows_idx
    while active.size:
        o = offs[active]
        c = active[:, None] + o
        bad = (c < 0) | (c >= n)
        # a repeated offset is invalid except for its first occurrence
        order = np.argsort(o, axis=1, kind="stable")
        so = np.take_along_axis(o, order, axis=1)
        dup_sorted = np.zeros_like(bad)
        dup_sorted[:, 1:] = so[:, 1:] == so[:, :-1]
        dup = np.zeros_like(bad)
        np.put_along_axis(dup, order, dup_sorted, axis=1)
        bad |= dup
        rows_bad = bad.any(axis=1)
        active, bad, o = active[rows_bad], bad[rows_bad], o[rows_bad]
        o[bad] = draw(int(bad.sum()))
        offs[active] = o
    cols = np.concatenate([rows_idx[:, None], rows_idx[:, None] + offs], axis=1)
    vals = np.empty((n, k + 1), dtype=np.float64)
    vals[:, 0] = rng.uniform(0.0, diag_max, size=n)
    vals[:, 1:] = rng.standard_normal((n, k)) / np.sqrt(nnz_per_row)
    order = np.argsort(cols, axis=1, kind="stable")
    cols = np.take_along_axis(cols, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    rowptr = np.arange(0, n * (k + 1) + 1, k + 1, dtype=np.int64)
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32 indices")
    return CSR(n, rowptr.astype(np.int32), cols.reshape(-1).astype(np.int32), vals.reshape(-1))


def band_with_rotations(n: int = 23560, nnz_per_row: int = 20, band: int = 200, seed: int = 2,
                        shift: float = 0.5, pair_frac: float = 0.02, mag: float = 12.0) -> CSR:
    """Nonsymmetric matrix with a complex spectrum and outlying conjugate
    pairs: ``random_banded`` (diagonal uniform on [0, 10]) plus ``shift`` on
    the diagonal, plus skew couplings +b, -b at (i, i+1), (i+1, i) for
    ``pair_frac * n / 2`` disjoint even i, b uniform on [mag/2, mag].  Each
    coupling moves a pair of eigenvalues far off the real axis, where a
    low-degree minimum residual polynomial is not small."""
    import scipy.sparse as sp
    base = random_banded(n, nnz_per_row, band, seed)
    S = base.to_scipy().tocoo()
    rng = np.random.default_rng([seed, 2])
    npairs = max(1, int(pair_frac * n / 2))
    i = rng.choice(n // 2, npairs, replace=False) * 2
    b = mag * rng.uniform(0.5, 1.0, npairs)
    d = np.arange(n)
    rows = np.concatenate([S.row, d, i, i + 1])
    cols = np.concatenate([S.col, d, i + 1, i])
    vals = np.concatenate([S.data, np.full(n, shift), b, -b])
    M = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    return CSR(n, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64))


def diag_csr(d: np.ndarray) -> CSR:
    d = np.asarray(d, dtype=np.float64)
    n = d.size
    return CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d.copy())


def dense_csr(A: np.ndarray, drop_zeros: bool = True) -> CSR:
    """CSR of a dense square array (small test matrices)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    if drop_zeros:
        r, c = np.nonzero(A)
    else:
        r, c = np.indices(A.shape).reshape(2, -1)
    return _from_coo(n, r.astype(np.int64), c.astype(np.int64), A[r, c])


def start_vectors(n: int, seed: int, count: int = 2) -> list[np.ndarray]:
    """Seeded N(0,1) vectors: first is the GMRES start vector b, second the
    Arnoldi start vector v0 (further draws for extra trials)."""
    rng = np.random.default_rng([seed, 1])
    return [rng.standard_normal(n) for _ in range(count)]


def stencil_nnz(dims) -> int:
    """Exact nnz of a 2*len(dims)+1 point stencil on a Dirichlet tensor grid."""
    n = int(np.prod(dims))
    nnz = n
    for d in dims:
        nnz += 2 * (n // d) * (d - 1)
    return nnz
