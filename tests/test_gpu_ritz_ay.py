"""GPU check of the Ritz test's A Y (section 4: the convergence test is
taken against A): the residuals the solver reports equal ||A x - mu x||
recomputed on the host from the returned vectors.

A Y runs four columns per sweep of the matrix when every row fits a
256-nonzero block and falls back to one pass per column when a row is
longer; both paths are covered, with column counts that leave a ragged last
group (2 nev = 10 and 6: groups of 4, 4, 2 and 4, 2).  Marked gpu; run on
an MI355X."""
import numpy as np
import pytest

from paper_1806_08020_amd import workloads as W

from .test_gpu_parity import dev, host

pytestmark = pytest.mark.gpu


def with_long_row(csr, row=5000, length=600, seed=3):
    """csr plus `length` small entries in one row (longer than a block)."""
    rng = np.random.default_rng(seed)
    coo = csr.to_scipy().tocoo()
    cols = rng.choice(np.setdiff1d(np.arange(csr.n), coo.col[coo.row == row]), length,
                      replace=False)
    return W._from_coo(csr.n, np.append(coo.row, np.full(length, row)), np.append(coo.col, cols),
                       np.append(coo.data, 1e-3 * rng.standard_normal(length)))


def host_residuals(csr, mu, X):
    S = csr.to_scipy()
    return np.array([np.linalg.norm(S @ X[t].real + 1j * (S @ X[t].imag) - mu[t] * X[t])
                     for t in range(mu.size)])


@pytest.mark.parametrize("long_row", [False, True])
@pytest.mark.parametrize("nev", [5, 3])
def test_reported_residuals_match_host(lib, long_row, nev):
    csr = W.convdiff_2d(100, 0.5)
    if long_row:
        csr = with_long_row(csr)
        assert np.diff(csr.rowptr).max() > 256
    b, v0 = W.start_vectors(csr.n, 21)
    A = lib.Matrix(csr)
    P = lib.Poly.build(A, 10, dev(b))
    r = lib.eigs(A, P, dev(v0), 30, 12, nev, rtol=1e-8, max_cycles=30, want_vectors=True)
    X = host(r.X)
    assert r.mu.size == nev
    assert np.all(np.abs(np.linalg.norm(X, axis=1) - 1) < 1e-12)
    res = host_residuals(csr, r.mu, X)
    assert np.allclose(res, r.resid, rtol=1e-6, atol=1e-14 * A.norm_inf), (res, r.resid)
