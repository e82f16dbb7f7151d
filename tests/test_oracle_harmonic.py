"""Pins of the oracle's harmonic restart (the harmonic Arnoldi variant that
section 4, Example 2 uses: harmonic Ritz vectors kept at each restart)."""
import numpy as np
import pytest

import oracle as O
from paper_1806_08020_amd import workloads as W

from .test_oracle_arnoldi import multiset_match


def _harmonic_values_of_block(Hbar, k, target):
    """Harmonic Ritz values of a Krylov-like decomposition op V_k = V_{k+1} Hbar
    with a full (k+1) x k block: with c its last row, the eigenvalues of
    H_k + (H_k - tau I)^{-T} c^T c (reducing to the standard formula when c is
    h e_k^T)."""
    Hk = Hbar[:k, :k]
    c = Hbar[k, :k]
    F = np.linalg.solve((Hk - target * np.eye(k)).T, np.eye(k))
    return np.linalg.eigvals(Hk + F @ np.outer(c, c))


def test_restart_relation_and_kept_harmonic_values():
    """After a harmonic restart the kept basis satisfies op V_kk = V_{kk+1} H
    with a full (kk+1) x kk block and V orthonormal, and the harmonic Ritz
    values of that block are the kept ones."""
    A = W.convdiff_2d(16, 0.6)
    mv = O.csr_matvec(A)
    b, v0 = W.start_vectors(A.n, 3)
    roots, _ = O.gmres_poly(mv, b, 6)
    op = lambda x: O.apply_poly(mv, roots, x)
    events = []
    O.thick_restart_arnoldi(op, mv, v0, 24, 10, 6, 0.0, 3, hook=lambda *a: events.append(a),
                            harmonic=True)
    cyc = [e for e in events if e[0] == "cycle"]
    rst = [e for e in events if e[0] == "restart"]
    assert len(rst) >= 2
    for (_, Vc, Hc, mc), (_, V, H, kk) in zip(cyc, rst):
        Vk1 = V[:, : kk + 1]
        assert np.allclose(Vk1.T @ Vk1, np.eye(kk + 1), atol=1e-12)
        R = np.column_stack([op(V[:, j]) for j in range(kk)]) - Vk1 @ H[: kk + 1, :kk]
        assert np.linalg.norm(R) <= 1e-10 * np.linalg.norm(H)
        theta, G, f = O.harmonic_projection(Hc[:mc, :mc], Hc[mc, mc - 1], 1.0)
        kept = theta[O.sort_ritz(theta, 1.0)][:kk]
        multiset_match(_harmonic_values_of_block(H[: kk + 1, :kk], kk, 1.0), kept, 1e-9)


def test_harmonic_values_reduce_to_ritz_values_without_residual():
    """h_{m+1,m} = 0 (an invariant subspace): harmonic and standard Ritz values
    coincide."""
    rng = np.random.default_rng(4)
    Hm = np.triu(rng.standard_normal((8, 8)), -1)
    theta, _, _ = O.harmonic_projection(Hm, 0.0, 1.0)
    multiset_match(theta, np.linalg.eigvals(Hm), 1e-12)


@pytest.mark.parametrize("N,bh,nev", [(50, 0.0, 10), (20, 0.5, 6)])
def test_harmonic_solve_closed_form(N, bh, nev):
    """Laplacian 50x50 and convection-diffusion 20x20 (beta*h = 0.5): the
    harmonic variant converges to the closed-form smallest eigenvalues."""
    A = W.laplacian_2d(N) if bh == 0.0 else W.convdiff_2d(N, bh)
    g = bh / 2
    i = np.arange(1, N + 1)
    lam = np.sort((4 - 2 * np.sqrt(1 - g * g) * np.cos(i[:, None] * np.pi / (N + 1))
                   - 2 * np.cos(i[None, :] * np.pi / (N + 1))).ravel())
    rng = np.random.default_rng([N, 1])
    b, v0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    res, _ = O.pp_eigs(A, b, v0, 30, 15, nev, d=10 if bh == 0 else 8, rtol=1e-10, max_cycles=200,
                       harmonic=True)
    assert res.converged
    assert np.allclose(np.sort(res.mu.real), lam[:nev], rtol=0, atol=1e-8)


def test_harmonic_dense_brute_force_with_pair():
    """Random nonsymmetric n = 300 with a complex pair near the origin: the
    harmonic variant returns the six eigenvalues of smallest magnitude."""
    rng = np.random.default_rng(1)
    n = 300
    lam = np.concatenate([rng.uniform(0.5, 10.0, n - 6), [0.11, 0.2, 0.27, 0.35]])
    X = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    D = np.diag(np.concatenate([lam[: n - 2], [0.0, 0.0]]))
    D[n - 2:, n - 2:] = [[0.3, 0.15], [-0.15, 0.3]]
    A = X @ D @ np.linalg.inv(X)
    csr = W.dense_csr(A, drop_zeros=False)
    ev = np.linalg.eigvals(A)
    ev = ev[np.lexsort((ev.imag, ev.real, np.abs(ev)))]
    b, v0 = W.start_vectors(n, 1)
    res, _ = O.pp_eigs(csr, b, v0, m=30, k=12, nev=6, d=6, rtol=1e-10, max_cycles=400, harmonic=True)
    assert res.converged
    multiset_match(res.mu, ev[:6], 1e-7)
    assert np.any(np.abs(res.mu.imag) > 0.1)


# ---------------------------------------------------------------- planted mistakes
import oracle.ppa_oracle as P  # noqa: E402


def _restart_plain_vnext(V, H, G, theta, f, k, m):
    # keeps v_{m+1} as the next vector, as the standard restart does
    return P.thick_restart(V, H, G, theta, k, m)


def _projection_untransposed(Hm, hm, target):
    m = Hm.shape[0]
    e = np.zeros(m)
    e[-1] = 1.0
    f = np.linalg.solve(Hm - target * np.eye(m), e)
    theta, G = np.linalg.eig(Hm + hm * hm * np.outer(f, e))
    return theta, G, f


@pytest.mark.parametrize("attr,fn", [("harmonic_restart", _restart_plain_vnext),
                                     ("harmonic_projection", _projection_untransposed)])
def test_harmonic_mutant_is_caught(attr, fn, monkeypatch):
    monkeypatch.setattr(P, attr, fn)
    monkeypatch.setattr(O, attr, fn)
    with pytest.raises(AssertionError):
        test_restart_relation_and_kept_harmonic_values()
