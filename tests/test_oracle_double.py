"""Pins of the oracle's double polynomial preconditioning (section 8)."""
import numpy as np

import oracle as O
from paper_1806_08020_amd import workloads as W


def test_composite_spectral_mapping_diagonal():
    """On a diagonal A, pi_2(tau(A)) v has entries v_i pi_2(tau(lambda_i)),
    tau = 1 - pi_1, evaluated as scalar products of the factors."""
    rng = np.random.default_rng(1)
    lam = np.sort(rng.uniform(0.05, 4.0, 200))
    A = W.diag_csr(lam)
    mv = O.csr_matvec(A)
    b = rng.standard_normal(200)
    r1, r2 = O.double_poly(mv, b, 4, 6)
    v = rng.standard_normal(200)
    y = O.apply_double(mv, r1, r2, v)
    p1 = np.array([np.prod(1 - l / r1) for l in lam]).real
    tau = 1 - p1
    p2 = np.array([np.prod(1 - t / r2) for t in tau]).real
    assert np.allclose(y, v * p2, rtol=1e-10, atol=1e-12 * np.abs(v).max())


def test_composite_is_one_at_zero_and_degree():
    """pi_2(tau(0)) = pi_2(0) = 1, and the composite has degree d1*d2: it
    uses exactly d1*d2 products with A per application."""
    rng = np.random.default_rng(2)
    A = W.convdiff_2d(12, 0.3)
    mv = O.csr_matvec(A)
    b = rng.standard_normal(A.n)
    r1, r2 = O.double_poly(mv, b, 3, 4)
    z = O.csr_matvec(W.diag_csr(np.zeros(5)))
    v = rng.standard_normal(5)
    assert np.allclose(O.apply_double(z, r1, r2, v), v)
    cnt = O.Counters()
    O.apply_double(mv, r1, r2, rng.standard_normal(A.n), cnt)
    assert cnt.mvps == 12


def test_second_polynomial_is_min_residual_on_tau():
    """pi_2 is the GMRES polynomial of tau(A) for b: pi_2(tau(A)) b is the
    least-squares residual over [tau b, tau^2 b, ...]."""
    rng = np.random.default_rng(3)
    A = W.convdiff_2d(10, 0.2)
    mv = O.csr_matvec(A)
    b = rng.standard_normal(A.n)
    r1, r2 = O.double_poly(mv, b, 3, 4)
    T = lambda x: O.tau_apply(mv, r1, x)
    cols = [T(b)]
    for _ in range(3):
        cols.append(T(cols[-1]))
    K = np.array(cols).T
    s = np.linalg.norm(K, axis=0)
    y, *_ = np.linalg.lstsq(K / s, b, rcond=None)
    res_ls = b - (K / s) @ y
    assert np.linalg.norm(O.apply_double(mv, r1, r2, b) - res_ls) <= 1e-8 * np.linalg.norm(b)


def test_double_poly_eigs_laplacian():
    """Double polynomial Arnoldi finds Laplacian eigenvalues (closed form)."""
    A = W.laplacian_2d(30, 31)
    b, v0 = W.start_vectors(A.n, 9)
    res, _ = O.pp_eigs(A, b, v0, m=20, k=10, nev=6, d1=4, d2=5, rtol=1e-8, max_cycles=60)
    assert res.converged
    i = np.arange(1, 31)[:, None]
    j = np.arange(1, 32)[None, :]
    lam = np.sort((4 - 2 * np.cos(i * np.pi / 31) - 2 * np.cos(j * np.pi / 32)).ravel())
    assert np.allclose(res.mu.real, lam[:6], rtol=1e-9)
