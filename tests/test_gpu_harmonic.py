"""GPU tests of the harmonic restart (the harmonic Arnoldi variant of section
4, Example 2): harmonic Ritz pairs eig(H_m + h^2 f e_m^T) with
(H_m - tau I)^T f = e_m, and a restart that keeps harmonic Ritz vectors plus
the shared residual direction v_{m+1} - h V_m f (a full (kk+1) x kk block)."""
import numpy as np
import pytest

import oracle as O
from paper_1806_08020_amd import workloads as W

from .test_oracle_arnoldi import multiset_match
from .test_gpu_shift import dev

pytestmark = pytest.mark.gpu


def closed_form(N, bh):
    g = bh / 2
    i = np.arange(1, N + 1)
    return np.sort((4 - 2 * np.sqrt(1 - g * g) * np.cos(i[:, None] * np.pi / (N + 1))
                    - 2 * np.cos(i[None, :] * np.pi / (N + 1))).ravel())


@pytest.mark.parametrize("N,bh,nev,d", [(50, 0.0, 10, 10), (20, 0.5, 6, 8)])
def test_harmonic_solve_closed_form(lib, N, bh, nev, d):
    """Laplacian 50x50 and convection-diffusion 20x20 (beta*h = 0.5) with a
    polynomial: the harmonic variant converges to the closed-form smallest
    eigenvalues, as the oracle's harmonic run does."""
    csr = W.laplacian_2d(N) if bh == 0.0 else W.convdiff_2d(N, bh)
    rng = np.random.default_rng([N, 1])
    b, v0 = rng.standard_normal(csr.n), rng.standard_normal(csr.n)
    A = lib.Matrix(csr)
    P = lib.Poly.build(A, d, dev(b))
    r = lib.eigs(A, P, dev(v0), 30, 15, nev, rtol=1e-10, max_cycles=200, harmonic=True)
    assert r.converged
    assert np.allclose(np.sort(r.mu.real), closed_form(N, bh)[:nev], rtol=0, atol=1e-8)
    assert np.all(r.resid <= 1e-10 * A.norm_inf)


def test_harmonic_trajectory_matches_oracle(lib):
    """Same operator (the oracle's roots), same start vector, three cycles of
    harmonic Arnoldi(24,10): after each cycle count the wanted harmonic Ritz
    values of pi(A), the Rayleigh quotients and the residuals match the
    oracle's (the restart block and the extra vector enter every later
    cycle, so a wrong restart shows here), and differ from the standard
    restart's.  Convection-diffusion 40x40, beta*h = 0.6, d = 3,
    Arnoldi(16,6): residuals fall from 1e-1 to 1e-6 over six cycles."""
    csr = W.convdiff_2d(40, 0.6)
    b, v0 = W.start_vectors(csr.n, 3)
    mv = O.csr_matvec(csr)
    roots, _ = O.gmres_poly(mv, b, 3)
    A = lib.Matrix(csr)
    P = lib.Poly.from_roots(roots)
    for cycles in (1, 3, 6):
        r = lib.eigs(A, P, dev(v0), 16, 6, 6, rtol=0.0, max_cycles=cycles, harmonic=True)
        o, _ = O.pp_eigs(csr, b, v0, 16, 6, 6, rtol=0.0, max_cycles=cycles, roots=roots,
                         harmonic=True)
        assert r.cycles == o.cycles == cycles
        multiset_match(r.nu, o.nu, 1e-9)
        multiset_match(r.mu, o.mu, 1e-9)
        assert np.allclose(np.sort(r.resid), np.sort(o.resid), rtol=1e-5, atol=1e-13)
        if cycles == 6:
            s = lib.eigs(A, P, dev(v0), 16, 6, 6, rtol=0.0, max_cycles=cycles)
            assert np.max(np.abs(np.sort(s.resid) - np.sort(r.resid))) > 1e-6


def test_harmonic_without_polynomial_targets_origin(lib):
    """Standard Arnoldi (no polynomial) with the harmonic restart, target 0:
    the smallest eigenvalues of a nonsymmetric matrix with a complex pair
    near the origin, against the dense eigenvalues (brute force)."""
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
    P = lib.Poly.build(A, 6, dev(b))
    r = lib.eigs(A, P, dev(v0), 30, 12, 6, rtol=1e-10, max_cycles=400, harmonic=True)
    assert r.converged
    multiset_match(r.mu, ev[:6], 1e-7)
    assert np.any(np.abs(r.mu.imag) > 0.1)
    r0 = lib.eigs(A, None, dev(v0), 40, 15, 5, rtol=1e-10, max_cycles=2000, harmonic=True)
    assert r0.converged
    multiset_match(r0.mu, ev[:5], 1e-7)


def test_harmonic_example2_standin_matches_oracle_counts(lib):
    """Example 2's comparison on a stand-in of its shape (n = 3000, 20
    nonzeros per row, outlying conjugate pairs; the degree-5 polynomial
    exceeds 1 in modulus on some eigenvalues): with the oracle's roots, the
    device's Ritz and harmonic runs converge to the oracle's eigenvalues in
    the oracle's cycle counts (within two), and the harmonic restart takes
    fewer cycles, as in the oracle."""
    csr = W.band_with_rotations(3000)
    b, v0 = W.start_vectors(csr.n, 10)
    roots, _ = O.gmres_poly(O.csr_matvec(csr), b, 5)
    A = lib.Matrix(csr)
    P = lib.Poly.from_roots(roots)
    cyc = {}
    for harm in (False, True):
        o, _ = O.pp_eigs(csr, b, v0, 50, 20, 15, rtol=1e-8, max_cycles=400, roots=roots, harmonic=harm)
        r = lib.eigs(A, P, dev(v0), 50, 20, 15, rtol=1e-8, max_cycles=400, harmonic=harm)
        assert o.converged and r.converged
        assert abs(r.cycles - o.cycles) <= 2, (harm, r.cycles, o.cycles)
        multiset_match(r.mu, o.mu, 1e-7)
        cyc[harm] = (r.cycles, o.cycles)
    assert cyc[True][0] < cyc[False][0] and cyc[True][1] < cyc[False][1]
