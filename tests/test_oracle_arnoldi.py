"""Pins of the oracle's thick-restarted Arnoldi on pi(A): closed-form
spectra, dense brute force, invariants of the Arnoldi relation and of the
restart, shift invariance at d = 1, and the paper's printed counts.  CPU only."""
import os

import numpy as np
import pytest

import oracle as O
from paper_1806_08020_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def lap_closed_form(nx, ny):
    i = np.arange(1, nx + 1)[:, None]
    j = np.arange(1, ny + 1)[None, :]
    return np.sort((4 - 2 * np.cos(i * np.pi / (nx + 1)) - 2 * np.cos(j * np.pi / (ny + 1))).ravel())


def convdiff_closed_form(N, bh):
    i = np.arange(1, N + 1)[:, None]
    j = np.arange(1, N + 1)[None, :]
    c = np.sqrt(1 - (bh / 2) ** 2)
    return np.sort((4 - 2 * c * np.cos(i * np.pi / (N + 1)) - 2 * np.cos(j * np.pi / (N + 1))).ravel())


def multiset_match(got, exact, tol):
    """Each returned value matches a distinct true eigenvalue (greedy)."""
    pool = list(exact)
    for g in got:
        k = int(np.argmin([abs(g - p) for p in pool]))
        assert abs(g - pool[k]) <= tol, (g, pool[k])
        pool.pop(k)


def test_config1_laplacian_closed_form():
    """50x50 Laplacian, d=10, Arnoldi(30,15), nev=10, rtol 1e-8: every
    returned eigenvalue is a closed-form eigenvalue 4-2cos(i pi/51)-2cos(j pi/51)
    (multiset sense: the spectrum has double eigenvalues)."""
    A = W.laplacian_2d(50)
    b, v0 = W.start_vectors(A.n, 1)
    res, _ = O.pp_eigs(A, b, v0, m=30, k=15, nev=10, d=10, rtol=1e-8, max_cycles=100)
    assert res.converged
    assert np.all(res.resid <= 1e-8 * O.infnorm(A))
    lam = lap_closed_form(50, 50)
    multiset_match(res.mu.real, lam[:30], 1e-10)
    assert np.all(np.abs(res.mu.imag) < 1e-12)
    # the smallest (simple) eigenvalue is always found
    assert abs(res.mu[0].real - lam[0]) < 1e-12


def test_laplacian_distinct_spectrum_exact():
    """50x51 grid: no repeated eigenvalues among the smallest, so the 10
    smallest are found exactly (eigenvalue error ~ r^2/gap)."""
    A = W.laplacian_2d(50, 51)
    b, v0 = W.start_vectors(A.n, 11)
    res, _ = O.pp_eigs(A, b, v0, m=30, k=15, nev=10, d=10, rtol=1e-8, max_cycles=100)
    assert res.converged
    lam = lap_closed_form(50, 51)
    assert np.allclose(res.mu.real, lam[:10], rtol=1e-10, atol=0)


def test_convdiff_closed_form_small():
    """Nonsymmetric convection-diffusion (beta h = 0.5) on a 20x20 grid:
    eigenvalues 4 - 2 sqrt(1-(beta h/2)^2) cos(i pi/21) - 2 cos(j pi/21)."""
    A = W.convdiff_2d(20, 0.5)
    b, v0 = W.start_vectors(A.n, 2)
    res, _ = O.pp_eigs(A, b, v0, m=30, k=12, nev=6, d=8, rtol=1e-10, max_cycles=200)
    assert res.converged
    lam = convdiff_closed_form(20, 0.5)
    multiset_match(res.mu.real, lam[:12], 1e-7)
    assert abs(res.mu[0] - lam[0]) < 1e-8


@pytest.mark.parametrize("seed,d", [(1, 6), (2, 4), (3, 10), (1, 0)])
def test_dense_brute_force(seed, d):
    """Random nonsymmetric n = 300 (complex eigenvalues present): the nev
    eigenvalues of smallest magnitude from dense eig."""
    rng = np.random.default_rng(seed)
    n = 300
    lam = np.concatenate([rng.uniform(0.5, 10.0, n - 6), [0.11, 0.2, 0.27, 0.35]])
    X = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    # block-diagonal rotation gives one complex pair near the origin
    D = np.diag(np.concatenate([lam[: n - 2], [0.0, 0.0]]))
    D[n - 2:, n - 2:] = [[0.3, 0.15], [-0.15, 0.3]]
    A = X @ D @ np.linalg.inv(X)
    csr = W.dense_csr(A, drop_zeros=False)
    ev = np.linalg.eigvals(A)
    ev = ev[np.lexsort((ev.imag, ev.real, np.abs(ev)))]
    b, v0 = W.start_vectors(n, seed)
    res, _ = O.pp_eigs(csr, b, v0, m=30, k=12, nev=6, d=d, rtol=1e-10, max_cycles=400)
    assert res.converged
    multiset_match(res.mu, ev[:6], 1e-7)
    assert np.any(np.abs(res.mu.imag) > 0.1)


def test_high_degree_entangles_large_eigenvalues():
    """Section 2 / section 6: a high-degree pi can map large eigenvalues of A
    near 1, and Arnoldi on pi(A) then returns them with small residuals.  The
    oracle reproduces the failure mode (seed 2, d = 10): converged, but not
    all returned values are among the smallest."""
    rng = np.random.default_rng(2)
    n = 300
    lam = np.concatenate([rng.uniform(0.5, 10.0, n - 6), [0.11, 0.2, 0.27, 0.35]])
    X = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    D = np.diag(np.concatenate([lam[: n - 2], [0.0, 0.0]]))
    D[n - 2:, n - 2:] = [[0.3, 0.15], [-0.15, 0.3]]
    A = X @ D @ np.linalg.inv(X)
    b, v0 = W.start_vectors(n, 2)
    res, _ = O.pp_eigs(W.dense_csr(A, drop_zeros=False), b, v0, m=30, k=12, nev=6, d=10,
                       rtol=1e-10, max_cycles=300)
    assert res.converged
    assert np.max(np.abs(res.mu)) > 5.0


def _collect(events):
    def hook(ev, V, H, j):
        events.append((ev, V, H, j))
    return hook


def test_arnoldi_relation_and_orthogonality():
    """pi(A) V_m = V_{m+1} Hbar_m and V^T V = I, in the first cycle and after
    restarts (thick restart keeps the relation: H_k = Q^T H_m Q plus the spike
    row h_{m+1,m} e_m^T Q)."""
    A = W.convdiff_2d(30, 0.3)
    b, v0 = W.start_vectors(A.n, 3)
    mv = O.csr_matvec(A)
    r, _ = O.gmres_poly(mv, b, 6)
    events = []
    O.pp_eigs(A, b, v0, m=20, k=8, nev=5, roots=r, rtol=1e-14, max_cycles=4, hook=_collect(events))
    assert sum(e[0] == "restart" for e in events) >= 2
    for ev, V, H, j in events:
        if ev == "cycle":
            m = j
            PV = np.array([O.apply_poly(mv, r, V[:, i]) for i in range(m)]).T
            assert np.linalg.norm(PV - V[:, : m + 1] @ H[: m + 1, :m]) <= 1e-11 * np.linalg.norm(PV)
            G = V[:, : m + 1].T @ V[:, : m + 1]
            assert np.linalg.norm(G - np.eye(m + 1)) <= 1e-12
        else:
            kk = j
            PV = np.array([O.apply_poly(mv, r, V[:, i]) for i in range(kk)]).T
            assert np.linalg.norm(PV - V[:, : kk + 1] @ H[: kk + 1, :kk]) <= 1e-9 * np.linalg.norm(PV)


def test_restart_keeps_wanted_ritz_values():
    """After a restart eig(H_k) equals the k kept Ritz values of H_m."""
    A = W.convdiff_2d(25, 0.6)
    b, v0 = W.start_vectors(A.n, 4)
    events = []
    O.pp_eigs(A, b, v0, m=24, k=10, nev=6, d=5, rtol=1e-15, max_cycles=3, hook=_collect(events))
    for a, c in zip(events, events[1:]):
        if a[0] == "cycle" and c[0] == "restart":
            Hm = a[2][: a[3], : a[3]]
            nu = np.linalg.eigvals(Hm)
            nu = nu[O.sort_ritz(nu)]
            kk = c[3]
            got = np.linalg.eigvals(c[2][:kk, :kk])
            multiset_match(got, nu[:kk], 1e-9 * max(1, np.abs(nu).max()))


def test_restart_with_pair_at_boundary():
    """A conjugate pair lands at positions k, k+1 of the sorted Ritz values:
    k is reduced to k-1 and the restarted basis still satisfies the Arnoldi
    relation (section 4 footnote: keep real arithmetic, do not split pairs)."""
    rng = np.random.default_rng(1)
    n = 300
    lam = np.concatenate([rng.uniform(0.5, 10.0, n - 6), [0.11, 0.2, 0.27, 0.35]])
    X = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    D = np.diag(np.concatenate([lam[: n - 2], [0.0, 0.0]]))
    D[n - 2:, n - 2:] = [[0.3, 0.15], [-0.15, 0.3]]
    A = X @ D @ np.linalg.inv(X)
    csr = W.dense_csr(A, drop_zeros=False)
    mv = O.csr_matvec(csr)
    b, v0 = W.start_vectors(n, 1)
    r, _ = O.gmres_poly(mv, b, 4)
    events = []
    O.pp_eigs(csr, b, v0, m=20, k=4, nev=3, roots=r, rtol=1e-30, max_cycles=2, hook=_collect(events))
    ev = [e for e in events if e[0] == "restart"]
    assert ev and ev[0][3] == 3
    _, V, H, kk = ev[0]
    PV = np.array([O.apply_poly(mv, r, V[:, i]) for i in range(kk)]).T
    assert np.linalg.norm(PV - V[:, : kk + 1] @ H[: kk + 1, :kk]) <= 1e-9 * np.linalg.norm(PV)
    assert np.linalg.norm(V[:, : kk + 1].T @ V[:, : kk + 1] - np.eye(kk + 1)) <= 1e-12


def test_keep_count_pair_rule():
    nu = np.array([0.9, 0.8 + 0.1j, 0.8 - 0.1j, 0.5])
    assert O.keep_count(nu, 2) == 1
    assert O.keep_count(nu, 3) == 3
    assert O.keep_count(nu, 1) == 1


def test_degree_one_shift_invariance():
    """Section 3: with d = 1 the preconditioned Krylov space equals the
    standard one, so the Ritz values satisfy nu = 1 - lambda/theta."""
    A = W.convdiff_2d(16, 0.4)
    b, v0 = W.start_vectors(A.n, 5)
    th = 3.7
    ev0, ev1 = [], []
    O.pp_eigs(A, b, v0, m=15, k=5, nev=3, d=0, rtol=1e-30, max_cycles=1,
              hook=lambda e, V, H, j: ev0.append(np.linalg.eigvals(H[:j, :j])))
    O.pp_eigs(A, b, v0, m=15, k=5, nev=3, roots=np.array([th + 0j]), rtol=1e-30, max_cycles=1,
              hook=lambda e, V, H, j: ev1.append(np.linalg.eigvals(H[:j, :j])))
    mapped = 1 - ev0[0] / th
    multiset_match(ev1[0], mapped, 1e-9)


def test_example6_one_cycle_counts():
    """Section 6, Example 6: diag(1..10000), Arnoldi(50,20), nev=15, d=50 with
    the damped start vector A b converges in one cycle with 2,565 mvps."""
    n, m, k, nev, d, cycles, mvps = np.loadtxt(os.path.join(GOLD, "example6_counts.txt")).astype(int)
    lam = np.arange(1, n + 1, dtype=float)
    A = W.diag_csr(lam)
    b, v0 = W.start_vectors(n, 6)
    res, _ = O.pp_eigs(A, lam * b, v0, m=m, k=k, nev=nev, d=d, rtol=1e-8, max_cycles=5)
    assert res.converged and res.cycles == cycles
    assert res.counters.mvps == mvps
    assert np.allclose(res.mu.real, np.arange(1, nev + 1), rtol=1e-7)


def test_counters_cgs2_and_poly():
    """Counting convention: a CGS2 step against j vectors costs 2j+1 dots
    and 4j+2 vops; a factor of pi(A) one mvp and one vop."""
    A = W.laplacian_2d(10)
    b, v0 = W.start_vectors(A.n, 7)
    res, r = O.pp_eigs(A, b, v0, m=10, k=4, nev=2, d=3, rtol=1e-30, max_cycles=1)
    c = res.counters
    gm_dots = sum(2 * j + 1 for j in range(1, 4))
    ar_dots = sum(2 * j + 1 for j in range(1, 11))
    assert c.dots == gm_dots + ar_dots
    assert c.mvps == 3 + 10 * 3 + 2
