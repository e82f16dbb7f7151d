"""Seeded input generators: shapes, nnz and structure of the synthetic
workloads (CPU only)."""
import numpy as np

from paper_1806_08020_amd import workloads as W


def test_stencil_nnz_counts():
    assert W.laplacian_2d(50).nnz == 12300 == W.stencil_nnz((50, 50))
    assert W.stencil_nnz((1000, 1000)) == 4_996_000
    assert W.stencil_nnz((160, 160, 160)) == 28_518_400
    assert W.convdiff_3d(12, 0.3).nnz == W.stencil_nnz((12, 12, 12))


def test_convdiff_couplings():
    N, bh = 6, 0.5
    A = W.convdiff_2d(N, bh).to_dense()
    i = 2 * N + 3
    assert A[i, i] == 4.0
    assert A[i, i - 1] == -1.0 - bh / 2 and A[i, i + 1] == -1.0 + bh / 2
    assert A[i, i - N] == -1.0 and A[i, i + N] == -1.0
    B = W.convdiff_3d(5, 0.3).to_dense()
    j = 25 + 5 + 2
    for s in (1, 5, 25):
        assert B[j, j - s] == -1.15 and B[j, j + s] == -0.85
    assert B[j, j] == 6.0


def test_csr_sorted_and_int32():
    for A in (W.laplacian_2d(7, 9), W.convdiff_3d(4, 0.1), W.random_banded(3000, 27, 500, seed=4)):
        assert A.rowptr.dtype == np.int32 and A.colind.dtype == np.int32
        for r in range(A.n):
            c = A.colind[A.rowptr[r]:A.rowptr[r + 1]]
            assert np.all(np.diff(c) > 0)


def test_random_banded_shape():
    n, band = 20000, 5000
    A = W.random_banded(n, 27, band, seed=4)
    assert A.nnz == 27 * n
    rows = np.repeat(np.arange(n), 27)
    off = A.colind.astype(np.int64) - rows
    assert np.all(np.abs(off) <= band)
    d = A.vals[off == 0]
    assert d.size == n and d.min() >= 0 and d.max() <= 10
    od = A.vals[off != 0]
    assert abs(od.std() - 1 / np.sqrt(27)) < 0.01
    B = W.random_banded(n, 27, band, seed=4)
    assert np.array_equal(A.colind, B.colind) and np.array_equal(A.vals, B.vals)


def test_start_vectors_seeded():
    b, v0 = W.start_vectors(100, 3)
    b2, v02 = W.start_vectors(100, 3)
    assert np.array_equal(b, b2) and np.array_equal(v0, v02) and not np.array_equal(b, v0)


def test_band_with_rotations_structure():
    """Random band plus a diagonal shift plus skew couplings on disjoint
    index pairs: A - base is shift*I + a block-diagonal skew part."""
    n = 3000
    A = W.band_with_rotations(n).to_scipy()
    B = W.random_banded(n, 20, 200, seed=2).to_scipy()
    D = (A - B).toarray()
    assert np.allclose(np.diag(D), 0.5)
    S = D - 0.5 * np.eye(n)
    assert np.allclose(S, -S.T)
    r, c = np.nonzero(np.abs(S) > 1e-9)
    assert np.all(np.abs(r - c) == 1) and np.all(np.minimum(r, c) % 2 == 0)
    assert r.size == 2 * int(0.02 * n / 2)
    v = np.abs(S[r, c])
    assert v.min() >= 6.0 and v.max() <= 12.0
    C1, C2 = W.band_with_rotations(n), W.band_with_rotations(n)
    assert np.array_equal(C1.colind, C2.colind) and np.array_equal(C1.vals, C2.vals)
    for row in range(n):
        assert np.all(np.diff(C1.colind[C1.rowptr[row]:C1.rowptr[row + 1]]) > 0)
