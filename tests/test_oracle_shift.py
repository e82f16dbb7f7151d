"""Pins of the oracle's shifted target (section 2 footnote: for eigenvalues
near mu, work with A - mu I) against closed-form spectra and an explicitly
shifted matrix."""
import numpy as np
import pytest

import oracle as O
from paper_1806_08020_amd import workloads as W


def lap_closed(N):
    i = np.arange(1, N + 1)
    return np.sort((4 - 2 * np.cos(i[:, None] * np.pi / (N + 1))
                    - 2 * np.cos(i[None, :] * np.pi / (N + 1))).ravel())


def nearest(lam, mu, k):
    return np.sort(lam[np.argsort(np.abs(lam - mu), kind="stable")][:k])


@pytest.mark.parametrize("shift", [8.5, -1.0])
def test_shifted_target_closed_form_laplacian(shift):
    """The 2-D Laplacian 50x50: with mu above the spectrum the solver returns
    its largest eigenvalues, with mu below its smallest, as multisets."""
    A = W.laplacian_2d(50)
    rng = np.random.default_rng([1, 1])
    b, v0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    res, _ = O.pp_eigs(A, b, v0, 30, 15, 10, d=10, rtol=1e-8, max_cycles=100, shift=shift)
    assert res.converged
    assert np.allclose(np.sort(res.mu.real), nearest(lap_closed(50), shift, 10), rtol=0, atol=1e-10)
    # returned in order of distance to the target
    assert np.all(np.diff(np.abs(res.mu - shift)) >= -1e-12)


def test_shifted_target_closed_form_convdiff():
    """Constant-coefficient convection-diffusion 20x20, beta*h = 0.5: the largest
    eigenvalues 4 - 2 sqrt(1 - g^2) cos(i pi/21) - 2 cos(j pi/21), g = 1/4
    (x-direction convection), found from mu = 9."""
    N, g = 20, 0.25
    A = W.convdiff_2d(N, 0.5)
    i = np.arange(1, N + 1)
    lam = np.sort((4 - 2 * np.sqrt(1 - g * g) * np.cos(i[:, None] * np.pi / (N + 1))
                   - 2 * np.cos(i[None, :] * np.pi / (N + 1))).ravel())
    rng = np.random.default_rng([2, 1])
    b, v0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    res, _ = O.pp_eigs(A, b, v0, 30, 12, 6, d=8, rtol=1e-10, max_cycles=200, shift=9.0)
    assert res.converged
    assert np.allclose(np.sort(res.mu.real), nearest(lam, 9.0, 6), rtol=0, atol=1e-8)


def test_shift_equals_explicitly_shifted_matrix():
    """Working on A with mu equals working on the CSR of A - mu I and adding mu
    to the returned eigenvalues (mu beyond the spectrum: an exterior target)."""
    A = W.convdiff_2d(18, 0.3)
    mu = 9.0
    S = A.to_scipy().tolil()
    S.setdiag(S.diagonal() - mu)
    S = S.tocsr()
    S.sort_indices()
    B = W.CSR(A.n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(float))
    rng = np.random.default_rng(9)
    b, v0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    r1, roots1 = O.pp_eigs(A, b, v0, 25, 10, 5, d=6, rtol=1e-10, max_cycles=60, shift=mu)
    r2, roots2 = O.pp_eigs(B, b, v0, 25, 10, 5, d=6, rtol=1e-10 * O.infnorm(A) / O.infnorm(B),
                           max_cycles=60)
    assert np.allclose(np.sort_complex(roots1), np.sort_complex(roots2), rtol=1e-9, atol=0)
    assert r1.converged and r2.converged
    assert np.allclose(np.sort_complex(r1.mu), np.sort_complex(r2.mu + mu), rtol=0, atol=1e-9)


# ---------------------------------------------------------------- planted mistakes
import oracle.ppa_oracle as P  # noqa: E402


def _pp_sign_flipped(csr, b, v0, m, k, nev, d=None, d1=None, d2=None, rtol=1e-8, max_cycles=100,
                     roots=None, hook=None, shift=0.0):
    return P.__dict__["_orig_pp"](csr, b, v0, m, k, nev, d=d, d1=d1, d2=d2, rtol=rtol,
                                  max_cycles=max_cycles, roots=roots, hook=hook, shift=-shift)


def _pp_test_on_shifted(csr, b, v0, m, k, nev, d=None, d1=None, d2=None, rtol=1e-8, max_cycles=100,
                        roots=None, hook=None, shift=0.0):
    # Rayleigh quotients taken on A - mu I and reported as such
    res, r = P.__dict__["_orig_pp"](csr, b, v0, m, k, nev, d=d, d1=d1, d2=d2, rtol=rtol,
                                    max_cycles=max_cycles, roots=roots, hook=hook, shift=shift)
    res.mu = res.mu - shift
    return res, r


@pytest.mark.parametrize("mut", [_pp_sign_flipped, _pp_test_on_shifted])
def test_shift_mutant_is_caught(mut, monkeypatch):
    monkeypatch.setitem(P.__dict__, "_orig_pp", P.pp_eigs)
    monkeypatch.setattr(P, "pp_eigs", mut)
    monkeypatch.setattr(O, "pp_eigs", mut)
    with pytest.raises(AssertionError):
        test_shifted_target_closed_form_laplacian(8.5)
