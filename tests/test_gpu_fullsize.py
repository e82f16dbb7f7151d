"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (matrix handles created with the default kernel choice,
which times the windowed variant against the plain one for large matrices).

* pi(A)v: whole output vectors against the FP64 oracle element by element
  (a CSR mat-vec at these sizes costs the oracle tens of milliseconds), with
  the same first-order rounding bound as the small-size tests;
* single fused passes in the launch configurations the solves run (column
  runs for the 3-D operator, the sliding window for the band matrix):
  bitwise equal to the plain kernel and within the bound of the host's
  CSR product;
* polynomial roots: the GPU's harmonic Ritz values against the oracle's own
  GMRES(d) run on the same seed vector;
* eigensolves: properties that hold at any size -- every returned pair's
  residual recomputed independently on the host from the returned vector,
  unit-norm vectors, reported residuals equal to the recomputed ones.

Workloads: 2-D convection-diffusion 1000x1000 (beta*h = 0.5, d = 50), 3-D
convection-diffusion 160^3 (beta*h = 0.3, double polynomial 10 x 20, FP32
pi(A)v), random banded n = 2e6 with 27 nonzeros per row within +-5000
(d = 100, FP32 pi(A)v).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1806_08020_amd import workloads as W

from .test_gpu_parity import EPS32, EPS64, chain_tol, dev, host, oracle_chain

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cd2():
    return W.convdiff_2d(1000, 0.5)


@pytest.fixture(scope="module")
def cd3():
    return W.convdiff_3d(160, 0.3)


@pytest.fixture(scope="module")
def band():
    return W.random_banded(2_000_000, 27, 5000, seed=4)


def match_roots(got, ref, rtol):
    """Every root of `got` has a partner in `ref` within rtol (relative), and
    the multisets have the same size and the same number of complex roots."""
    assert got.size == ref.size
    assert np.sum(got.imag != 0) == np.sum(ref.imag != 0)
    for z in got:
        assert np.min(np.abs(ref - z)) <= rtol * abs(z), z


def host_residuals(csr, mu, X):
    """||A x - mu x|| for each returned pair, from the host copy of x."""
    S = csr.to_scipy()
    out = []
    for t in range(mu.size):
        x = X[t]
        out.append(np.linalg.norm(S @ x.real + 1j * (S @ x.imag) - mu[t] * x))
    return np.array(out)


def test_cd2_full_roots_and_apply(lib, cd2):
    """n = 1e6, d = 50, FP64: roots against the oracle's GMRES(50) on the same
    b; pi(A)v on the GPU's roots against the oracle factor by factor."""
    b, v0 = W.start_vectors(cd2.n, 2)
    mv = O.csr_matvec(cd2)
    A = lib.Matrix(cd2)
    P = lib.Poly.build(A, 50, dev(b))
    roots = P.roots()
    oroots, _ = O.gmres_poly(mv, b, 50)
    match_roots(roots, oroots, 1e-9)
    y = host(lib.apply(A, P, dev(v0)))
    ref, g = oracle_chain(mv, roots, v0)
    err = np.max(np.abs(y - ref))
    assert err <= chain_tol(cd2, roots, g, EPS64), err


def test_cd3_full_double_poly_apply_fp32(lib, cd3):
    """n = 4.1e6, double polynomial 10 x 20 built on the GPU: pi_2(tau(A)) v
    in FP32 (values and vectors) and in FP64 against the FP64 oracle."""
    b, v0 = W.start_vectors(cd3.n, 3)
    mv = O.csr_matvec(cd3)
    A = lib.Matrix(cd3, want_f32=True)
    P = lib.Poly.build_double(A, 10, 20, dev(b))
    assert P.is_double and P.d1 == 10 and P.degree == 20
    r1, r2 = P.roots(1), P.roots(2)
    tau = lambda x: O.tau_apply(mv, r1, x)
    ref, g = oracle_chain(tau, r2, v0)
    tol = chain_tol(cd3, r1, g, EPS64) * len(r2) * 4
    y = host(lib.apply(A, P, dev(v0)))
    assert np.max(np.abs(y - ref)) <= tol
    y32 = host(lib.apply(A, P, dev(v0, torch.float32), precision="f32")).astype(float)
    assert np.max(np.abs(y32 - ref)) <= tol * (EPS32 / EPS64) * 2


def test_band_full_apply_fp32_and_fp64(lib, band):
    """n = 2e6, 27 nonzeros per row, d = 100: pi(A)v in FP32 (the kernel the
    matrix handle selected at creation) and FP64 against the oracle."""
    b, v0 = W.start_vectors(band.n, 4)
    mv = O.csr_matvec(band)
    A = lib.Matrix(band, want_f32=True)
    P = lib.Poly.build(A, 100, dev(b))
    roots = P.roots()
    ref, g = oracle_chain(mv, roots, v0)
    tol = chain_tol(band, roots, g, EPS64)
    y = host(lib.apply(A, P, dev(v0)))
    assert np.max(np.abs(y - ref)) <= tol
    y32 = host(lib.apply(A, P, dev(v0, torch.float32), precision="f32")).astype(float)
    assert np.max(np.abs(y32 - ref)) <= tol * (EPS32 / EPS64) * 2


def _check_pass(csr, run, run_ref, seed):
    """One fused pass, out = alpha x + beta A u, through `run` and through
    `run_ref` (each called as f(alpha, x, beta, u) on device vectors): the
    two are bitwise equal (same products, same summation order) and within
    the first-order bound of the host's FP64 CSR product.  Cases: a real
    root's pass (x is the gathered vector itself) and a conjugate pair's
    second pass (x and u distinct)."""
    rng = np.random.default_rng(seed)
    u, x = rng.standard_normal(csr.n), rng.standard_normal(csr.n)
    S = csr.to_scipy()
    Su, aSu = S @ u, abs(S) @ np.abs(u)
    nnzr = int(np.diff(csr.rowptr).max())
    ut = dev(u)
    for alpha, xv, beta in ((1.0, None, -0.3), (0.7, x, -1.3)):
        xt = ut if xv is None else dev(xv)
        y = run(alpha, xt, beta, ut)
        y0 = run_ref(alpha, xt, beta, ut)
        assert torch.equal(y, y0)
        xh = u if xv is None else xv
        ref = alpha * xh + beta * Su
        scale = abs(alpha) * np.abs(xh) + abs(beta) * aSu
        assert np.all(np.abs(host(y) - ref) <= (nnzr + 4) * EPS64 * scale)


def test_c3_headline_pass_in_the_benchmark_configuration(lib, cd3):
    """The headline pass as the benchmark times it: n = 4.1e6, FP64, column
    runs staged in LDS, non-temporal matrix loads, 2048 nonzeros per block;
    against the same kernel gathering from memory and the host's product."""
    A = lib.Matrix(cd3, window="runs")
    A.set_cache_policy("stream")
    A.set_spmv_blocks(2048)
    on, nb = A.spmv_runs("f64")
    assert on and nb >= 0.99 * A.nblocks
    assert A.cache_policy("f64") == "stream" and A.spmv_blocks("f64") == 2048

    def with_runs(flag):
        def run(alpha, x, beta, u):
            A.set_spmv_runs(flag)
            return lib.fused_spmv(A, alpha, x, beta, u)
        return run
    _check_pass(cd3, with_runs(True), with_runs(False), 31)


def test_band_full_sliding_window_pass(lib, band):
    """The banded matrix's FP64 pass as its solve runs it (n = 2e6, the
    sliding-window kernel, one 1024-thread block per CU), against the plain
    kernel and the host's product."""
    Ar = lib.Matrix(band, window="ring")
    Ap = lib.Matrix(band, window="off")
    assert Ar.spmv_variant("f64") == "ring" and Ap.spmv_variant("f64") == "plain"
    _check_pass(band, lambda a, x, b, u: lib.fused_spmv(Ar, a, x, b, u),
                lambda a, x, b, u: lib.fused_spmv(Ap, a, x, b, u), 32)


def test_cd2_full_eigs_fp64_properties(lib, cd2):
    """The benchmark's FP64 solve: d = 50, Arnoldi(50,25), nev = 20, rtol 1e-8."""
    b, v0 = W.start_vectors(cd2.n, 2)
    A = lib.Matrix(cd2)
    P = lib.Poly.build(A, 50, dev(b))
    r = lib.eigs(A, P, dev(v0), 50, 25, 20, rtol=1e-8, max_cycles=40, want_vectors=True)
    assert r.nconv == 20 and r.converged
    X = host(r.X)
    assert np.all(np.abs(np.linalg.norm(X, axis=1) - 1) < 1e-12)
    res = host_residuals(cd2, r.mu, X)
    assert np.all(res <= 1e-8 * A.norm_inf * 1.001), res.max() / A.norm_inf
    assert np.allclose(res, r.resid, rtol=1e-6, atol=1e-14 * A.norm_inf)
    # complex values come in conjugate pairs; the cut at nev may leave the
    # partner of the last (largest modulus) value outside the returned set
    cpx = r.mu[r.mu.imag != 0]
    for z in cpx:
        assert np.min(np.abs(cpx - np.conj(z))) <= 1e-14 or abs(z) >= np.abs(r.mu).max() * (1 - 1e-12), z


def test_cd3_full_eigs_mixed_properties(lib, cd3):
    """The benchmark's mixed-precision solve: FP32 pi(A)v, FP64 everything else
    and the closing FP64 pass; every returned pair meets rtol in FP64."""
    b, v0 = W.start_vectors(cd3.n, 3)
    A = lib.Matrix(cd3, want_f32=True)
    P = lib.Poly.build_double(A, 10, 20, dev(b))
    r = lib.eigs(A, P, dev(v0), 40, 20, 15, rtol=1e-8, max_cycles=20, precision="mixed",
                 want_vectors=True)
    assert r.nconv == 15 and r.converged
    assert r.fp32_cycles >= 1
    X = host(r.X)
    res = host_residuals(cd3, r.mu, X)
    assert np.all(res <= 1e-8 * A.norm_inf * 1.001), res.max() / A.norm_inf
    assert np.allclose(res, r.resid, rtol=1e-6, atol=1e-14 * A.norm_inf)


def test_band_full_eigs_reported_residuals(lib, band):
    """One restart cycle of the benchmark's mixed solve on the banded matrix
    (an interior problem that needs many cycles): the residuals it reports
    for its current Ritz pairs equal the host-recomputed ones."""
    b, v0 = W.start_vectors(band.n, 4)
    A = lib.Matrix(band, want_f32=True)
    P = lib.Poly.build(A, 100, dev(b))
    r = lib.eigs(A, P, dev(v0), 60, 15, 10, rtol=1e-8, max_cycles=1, precision="mixed",
                 want_vectors=True)
    assert r.cycles == 1
    X = host(r.X)
    assert np.all(np.abs(np.linalg.norm(X, axis=1) - 1) < 1e-12)
    res = host_residuals(band, r.mu, X)
    assert np.allclose(res, r.resid, rtol=1e-6, atol=1e-14 * A.norm_inf)


def test_cd2_full_harmonic_properties(lib, cd2):
    """The benchmark's operator with the harmonic restart (d = 50,
    Arnoldi(50,25), nev = 20): converged, every returned pair's residual
    recomputed on the host within rtol and equal to the reported one."""
    b, v0 = W.start_vectors(cd2.n, 2)
    A = lib.Matrix(cd2)
    P = lib.Poly.build(A, 50, dev(b))
    r = lib.eigs(A, P, dev(v0), 50, 25, 20, rtol=1e-8, max_cycles=40, harmonic=True, want_vectors=True)
    assert r.converged and r.nconv == 20
    X = host(r.X)
    res = host_residuals(cd2, r.mu, X)
    assert np.all(res <= 1e-8 * A.norm_inf * 1.001)
    assert np.allclose(res, r.resid, rtol=1e-6, atol=1e-14 * A.norm_inf)


def _closed_3d(N, bh, M=14):
    """Eigenvalues of the h^2-scaled 3-D operator -Lap u + beta (u_x + u_y +
    u_z) on N^3 (the same factor on each axis: eigenvalues of permuted index
    triples coincide exactly), lambda = 6 - 2 sqrt(1 - b^2) sum cos(i pi/(N+1)),
    b = beta h / 2, for the smallest indices (i, j, k < M), with each one's
    condition number: the product of the 1-D factors' ||D q_i|| ||D^-1 q_i|| /
    ||q_i||^2, D = diag(rho^k), rho = sqrt((1+b)/(1-b))."""
    b = 0.5 * bh
    k = np.arange(1, N + 1)
    th = k * np.pi / (N + 1)
    D = np.sqrt((1 + b) / (1 - b)) ** k
    kap = np.array([np.linalg.norm(D * np.sin(i * th)) * np.linalg.norm(np.sin(i * th) / D)
                    / (np.sin(i * th) @ np.sin(i * th)) for i in range(1, M + 1)])
    f = -2 * np.sqrt(1 - b * b) * np.cos(th[:M])
    I, J, K = np.meshgrid(np.arange(M), np.arange(M), np.arange(M), indexing="ij")
    lam = (6 + f[I] + f[J] + f[K]).ravel()
    kk = (kap[I] * kap[J] * kap[K]).ravel()
    o = np.argsort(lam)
    return lam[o], kk[o]


@pytest.mark.parametrize("bh", [0.02, 0.05])
def test_c3_grid_closed_form_eigenvalues(lib, bh):
    """The headline's grid (160^3), solve and polynomial (double 10 x 20,
    Arnoldi(40,20), nev = 15, FP64) with a convection weak enough that the
    closed form pins every eigenvalue: each returned value lies within
    2 kappa r of a closed-form eigenvalue (first order for a diagonalizable
    matrix, r its residual), and no eigenvalue is claimed more often than its
    multiplicity (1, 3 or 6 on this grid)."""
    csr = W.convdiff_3d(160, bh)
    b, v0 = W.start_vectors(csr.n, 3)
    A = lib.Matrix(csr)
    P = lib.Poly.build_double(A, 10, 20, dev(b))
    r = lib.eigs(A, P, dev(v0), 40, 20, 15, rtol=1e-8, max_cycles=12)
    print(f"160^3 beta*h={bh}: cycles {r.cycles}, converged {r.converged}", flush=True)
    assert r.converged and r.nconv == 15
    lam, kap = _closed_3d(160, bh)
    claimed = {}
    for mu, res in zip(r.mu, r.resid):
        assert res <= 1e-8 * A.norm_inf
        t = int(np.argmin(np.abs(lam - mu.real)))
        assert abs(mu - lam[t]) <= 2.0 * kap[t] * res + 1e-14 * A.norm_inf, (mu, lam[t])
        mult = int(np.sum(np.abs(lam - lam[t]) <= 1e-13))
        key = round(float(lam[t]), 12)
        claimed[key] = claimed.get(key, 0) + 1
        assert claimed[key] <= mult
    # the smallest eigenvalue is simple and always among those returned
    assert np.min(np.abs(r.mu - lam[0])) <= 2.0 * kap[0] * r.max_resid + 1e-14 * A.norm_inf


def test_c3_grid_closed_form_eigenvalues_mixed(lib):
    """The same pin for the mixed-precision solve (FP32 pi(A)v, the closing
    FP64 Rayleigh-Ritz pass, FP64 cycles as needed) at beta*h = 0.02 on the
    headline's grid: every returned eigenvalue within 2 kappa r of a
    closed-form one, multiplicities respected, at least one FP32 cycle."""
    bh = 0.02
    csr = W.convdiff_3d(160, bh)
    b, v0 = W.start_vectors(csr.n, 3)
    A = lib.Matrix(csr, want_f32=True)
    P = lib.Poly.build_double(A, 10, 20, dev(b))
    r = lib.eigs(A, P, dev(v0), 40, 20, 15, rtol=1e-8, max_cycles=12, precision="mixed")
    print(f"160^3 beta*h={bh} mixed: cycles {r.cycles}, fp32 cycles {r.fp32_cycles}", flush=True)
    assert r.converged and r.nconv == 15 and r.fp32_cycles >= 1
    lam, kap = _closed_3d(160, bh)
    claimed = {}
    for mu, res in zip(r.mu, r.resid):
        assert res <= 1e-8 * A.norm_inf
        t = int(np.argmin(np.abs(lam - mu.real)))
        assert abs(mu - lam[t]) <= 2.0 * kap[t] * res + 1e-14 * A.norm_inf, (mu, lam[t])
        mult = int(np.sum(np.abs(lam - lam[t]) <= 1e-13))
        key = round(float(lam[t]), 12)
        claimed[key] = claimed.get(key, 0) + 1
        assert claimed[key] <= mult


def test_c2_grid_laplacian_closed_form_eigenvalues(lib):
    """The 2-D workload's grid (1000 x 1000) and solve (d = 50, Arnoldi(50,25),
    nev = 20, FP64) on the Laplacian, the case whose closed form pins every
    value at this size (with convection the eigenvalue condition numbers grow
    as rho^N and no closed-form bound stays useful): each returned value lies
    within r^2 / gap of a closed-form eigenvalue (symmetric matrix, r its
    residual, gap the distance to the next distinct eigenvalue), no value is
    claimed more often than its multiplicity (2 for i != j), and the smallest
    eigenvalue (simple) is found."""
    N = 1000
    csr = W.laplacian_2d(N)
    b, v0 = W.start_vectors(csr.n, 2)
    A = lib.Matrix(csr)
    P = lib.Poly.build(A, 50, dev(b))
    r = lib.eigs(A, P, dev(v0), 50, 25, 20, rtol=1e-8, max_cycles=40)
    print(f"Laplacian {N}^2: cycles {r.cycles}, converged {r.converged}, max resid {r.max_resid:.2e}", flush=True)
    assert r.converged and r.nconv == 20
    M = 40
    th = np.arange(1, M + 1) * np.pi / (N + 1)
    f = 2 - 2 * np.cos(th)
    lam = (f[:, None] + f[None, :]).ravel()
    distinct = np.unique(np.round(lam, 13))
    claimed = {}
    for mu, res in zip(r.mu, r.resid):
        assert abs(mu.imag) <= 1e-14 * A.norm_inf
        u = int(np.argmin(np.abs(distinct - mu.real)))
        gap = np.min(np.abs(np.delete(distinct, u) - distinct[u]))
        bound = res * res / gap + 1e-14 * A.norm_inf
        assert abs(mu.real - distinct[u]) <= bound, (mu, distinct[u], bound)
        mult = int(np.sum(np.abs(lam - distinct[u]) <= 1e-12))
        claimed[u] = claimed.get(u, 0) + 1
        assert claimed[u] <= mult, (distinct[u], mult)
    assert 0 in claimed
