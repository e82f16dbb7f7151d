"""GPU tests of the low-synchronisation Gram-Schmidt (PPA_FLAG_LOWSYNC: the
reorthogonalisation of step j-1 delayed and merged with the projection of
step j, two passes over the basis per step) against the oracle's
``arnoldi_extend_dcgs2`` and against closed forms."""
import numpy as np
import pytest

import oracle as O
from paper_1806_08020_amd import workloads as W

from .test_gpu_parity import dev, host, lap_closed
from .test_gpu_fullsize import host_residuals
from .test_oracle_arnoldi import multiset_match

pytestmark = pytest.mark.gpu


def test_lowsync_laplacian_counters_and_values(lib):
    """50x50 Laplacian, d = 10, Arnoldi(30,15), nev = 10: closed-form values,
    the oracle's delayed-form values to 1e-10 relative, its cycle count, and
    the same mvps / dots / vops (the library excludes the polynomial build)."""
    csr = W.laplacian_2d(50)
    b, v0 = W.start_vectors(csr.n, 1)
    ores, oroots = O.pp_eigs(csr, b, v0, m=30, k=15, nev=10, d=10, rtol=1e-8, max_cycles=100,
                             ortho="dcgs2")
    A = lib.Matrix(csr)
    P = lib.Poly.from_roots(oroots)
    r = lib.eigs(A, P, dev(v0), 30, 15, 10, rtol=1e-8, max_cycles=100, lowsync=True, want_vectors=True)
    assert r.converged and r.nconv == 10 and r.cycles == ores.cycles
    lam = lap_closed(50, 50)
    for mu in r.mu:
        assert abs(mu.imag) < 1e-12 and np.min(np.abs(lam - mu.real)) <= 1e-10 * abs(mu.real)
    assert np.allclose(np.sort(r.mu.real), np.sort(ores.mu.real), rtol=1e-10, atol=0)
    assert (r.mvps, r.dots, r.vops) == (ores.counters.mvps - 10, ores.counters.dots - sum(
        2 * j + 1 for j in range(1, 11)), ores.counters.vops - sum(4 * j + 2 for j in range(1, 11)))
    X = host(r.X)
    res = host_residuals(csr, r.mu, X)
    assert np.all(res <= 1e-8 * A.norm_inf * 1.01)


@pytest.mark.parametrize("side", [40, 39])
def test_lowsync_trajectory_matches_oracle_and_default(lib, side):
    """Convection-diffusion 40x40 and 39x39 (beta*h = 0.6; even and odd n,
    so both the row-pair and the single-row kernels run), d = 3,
    Arnoldi(16,6), the oracle's roots: after 1, 3 and 6 cycles the wanted
    Ritz values of pi(A), the Rayleigh quotients and the residuals equal the
    oracle's delayed-form run and the device's default Gram-Schmidt run (the
    same Arnoldi decomposition in exact arithmetic; restarts included)."""
    csr = W.convdiff_2d(side, 0.6)
    b, v0 = W.start_vectors(csr.n, 3)
    roots, _ = O.gmres_poly(O.csr_matvec(csr), b, 3)
    A = lib.Matrix(csr)
    P = lib.Poly.from_roots(roots)
    for cycles in (1, 3, 6):
        r = lib.eigs(A, P, dev(v0), 16, 6, 6, rtol=0.0, max_cycles=cycles, lowsync=True)
        d = lib.eigs(A, P, dev(v0), 16, 6, 6, rtol=0.0, max_cycles=cycles)
        o, _ = O.pp_eigs(csr, b, v0, 16, 6, 6, rtol=0.0, max_cycles=cycles, roots=roots, ortho="dcgs2")
        assert r.cycles == o.cycles == cycles
        for other in (o.nu, d.nu):
            multiset_match(r.nu, other, 1e-9)
        for other in (o.mu, d.mu):
            multiset_match(r.mu, other, 1e-9)
        assert np.allclose(np.sort(r.resid), np.sort(o.resid), rtol=1e-5, atol=1e-13)


def test_lowsync_no_polynomial_and_harmonic(lib):
    """Dense nonsymmetric n = 300 with a complex pair near 0: standard Arnoldi
    (no polynomial) and the harmonic restart with a polynomial, both with the
    delayed Gram-Schmidt, reach the brute-force eigenvalues."""
    rng = np.random.default_rng(1)
    n = 300
    lam = np.concatenate([rng.uniform(0.5, 10.0, n - 6), [0.11, 0.2, 0.27, 0.35]])
    X = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    D = np.diag(np.concatenate([lam[: n - 2], [0.0, 0.0]]))
    D[n - 2:, n - 2:] = [[0.3, 0.15], [-0.15, 0.3]]
    Ad = X @ D @ np.linalg.inv(X)
    csr = W.dense_csr(Ad, drop_zeros=False)
    ev = np.linalg.eigvals(Ad)
    ev = ev[np.lexsort((ev.imag, ev.real, np.abs(ev)))]
    b, v0 = W.start_vectors(n, 1)
    A = lib.Matrix(csr)
    r0 = lib.eigs(A, None, dev(v0), 40, 15, 5, rtol=1e-10, max_cycles=2000, lowsync=True)
    assert r0.converged
    multiset_match(r0.mu, ev[:5], 1e-7)
    P = lib.Poly.build(A, 6, dev(b))
    rh = lib.eigs(A, P, dev(v0), 30, 12, 6, rtol=1e-10, max_cycles=400, harmonic=True, lowsync=True)
    assert rh.converged
    multiset_match(rh.mu, ev[:6], 1e-7)


def test_lowsync_breakdown(lib):
    """A = diag with five distinct values: the Krylov space is invariant after
    five steps; the delayed form stops the cycle there and returns the five
    eigenvalues."""
    d = np.repeat([1.0, 2.0, 3.5, 5.0, 8.0], 40)
    csr = W.diag_csr(d)
    rng = np.random.default_rng(2)
    A = lib.Matrix(csr)
    r = lib.eigs(A, None, dev(rng.standard_normal(d.size)), 12, 6, 5, rtol=1e-10, max_cycles=3,
                 lowsync=True)
    assert np.allclose(np.sort(r.mu.real), [1, 2, 3.5, 5, 8], rtol=0, atol=1e-10)


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_lowsync_full_size_convdiff(lib, prec):
    """The benchmark's operator (convection-diffusion 1000x1000, d = 50,
    Arnoldi(50,25), nev = 20, rtol 1e-8) with the delayed form: converged,
    every returned pair's residual recomputed on the host within rtol and
    equal to the reported one."""
    csr = W.convdiff_2d(1000, 0.5)
    b, v0 = W.start_vectors(csr.n, 2)
    A = lib.Matrix(csr, want_f32=(prec == "mixed"))
    P = lib.Poly.build(A, 50, dev(b))
    r = lib.eigs(A, P, dev(v0), 50, 25, 20, rtol=1e-8, max_cycles=40, precision=prec, lowsync=True,
                 want_vectors=True)
    assert r.converged and r.nconv == 20
    X = host(r.X)
    res = host_residuals(csr, r.mu, X)
    assert np.all(res <= 1e-8 * A.norm_inf * 1.001)
    assert np.allclose(res, r.resid, rtol=1e-6, atol=1e-14 * A.norm_inf)


def test_lowsync_gmres_roots(lib):
    """GMRES(d) with the delayed Gram-Schmidt: the harmonic Ritz values match
    the oracle's GMRES (immediate reorthogonalisation; the same Hbar in exact
    arithmetic) to 1e-9 relative -- convection-diffusion 30x30 with beta*h
    = 1.6 (complex roots), d = 14, and the benchmark's operator at d = 50."""
    for csr, d, seed in ((W.convdiff_2d(30, 1.6), 14, 12), (W.convdiff_2d(1000, 0.5), 50, 2)):
        b, _ = W.start_vectors(csr.n, seed)
        A = lib.Matrix(csr)
        P = lib.Poly.build(A, d, dev(b), lowsync=True)
        ref, _ = O.gmres_poly(O.csr_matvec(csr), b, d)
        got = P.roots()
        assert got.size == ref.size and np.sum(got.imag != 0) == np.sum(ref.imag != 0)
        for z in got:
            assert np.min(np.abs(ref - z)) <= 1e-9 * abs(z), z


def test_lowsync_safeguard_decisions(lib):
    """Example 6 (A = diag(1..10000), d = 50) with the Ideal-Order-Condition
    heuristic: the delayed form takes the same decisions (degree, damping,
    attempts, held) as the immediate form, and two start vectors give the
    same roots both ways."""
    csr = W.diag_csr(np.arange(1, 10001, dtype=float))
    rng = np.random.default_rng([6, 1])
    b = dev(rng.standard_normal(csr.n))
    b2 = dev(rng.standard_normal(csr.n))
    A = lib.Matrix(csr)
    _, i0 = lib.Poly.build_ex(A, 50, b, test=(50, 20, 15))
    _, i1 = lib.Poly.build_ex(A, 50, b, test=(50, 20, 15), lowsync=True)
    assert i0 == i1
    P0, _ = lib.Poly.build_ex(A, 12, b, b2=b2)
    P1, _ = lib.Poly.build_ex(A, 12, b, b2=b2, lowsync=True)
    r0, r1 = P0.roots(), P1.roots()
    for z in r1:
        assert np.min(np.abs(r0 - z)) <= 1e-9 * abs(z)
