"""GPU tests of the shifted target (section 2 footnote: A - mu I): the
polynomial is built for and applied to A - mu I with the shift folded into the
fused passes' coefficients; Ritz values are tested and returned for A."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1806_08020_amd import workloads as W

from .test_gpu_parity import EPS32, EPS64, host

pytestmark = pytest.mark.gpu


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.asarray(x)).to(device="cuda", dtype=dtype)


def lap_closed(N):
    i = np.arange(1, N + 1)
    return np.sort((4 - 2 * np.cos(i[:, None] * np.pi / (N + 1))
                    - 2 * np.cos(i[None, :] * np.pi / (N + 1))).ravel())


def nearest(lam, mu, k):
    return np.sort(lam[np.argsort(np.abs(lam - mu), kind="stable")][:k])


def shifted_mv(csr, mu):
    mv = O.csr_matvec(csr)
    return lambda x: mv(x) - mu * x


@pytest.mark.parametrize("shift", [8.5, -1.0])
def test_shifted_solve_laplacian_closed_form(lib, shift):
    csr = W.laplacian_2d(50)
    rng = np.random.default_rng([1, 1])
    b, v0 = rng.standard_normal(csr.n), rng.standard_normal(csr.n)
    A = lib.Matrix(csr)
    P, info = lib.Poly.build_ex(A, 10, dev(b), shift=shift)
    assert P.shift == shift
    ref, _ = O.gmres_poly(shifted_mv(csr, shift), b, 10)
    for z in P.roots():
        assert np.min(np.abs(ref - z)) <= 1e-9 * abs(z)
    r = lib.eigs(A, P, dev(v0), 30, 15, 10, rtol=1e-8, max_cycles=100)
    assert r.converged
    assert np.allclose(np.sort(r.mu.real), nearest(lap_closed(50), shift, 10), rtol=0, atol=1e-10)
    assert np.all(np.diff(np.abs(r.mu - shift)) >= -1e-12)
    ores, _ = O.pp_eigs(csr, b, v0, 30, 15, 10, d=10, rtol=1e-8, max_cycles=100, shift=shift)
    assert np.allclose(np.sort(r.mu.real), np.sort(ores.mu.real), rtol=0, atol=1e-10)


def test_shifted_solve_convdiff_closed_form(lib):
    N, g = 20, 0.25
    csr = W.convdiff_2d(N, 0.5)
    i = np.arange(1, N + 1)
    lam = np.sort((4 - 2 * np.sqrt(1 - g * g) * np.cos(i[:, None] * np.pi / (N + 1))
                   - 2 * np.cos(i[None, :] * np.pi / (N + 1))).ravel())
    rng = np.random.default_rng([2, 1])
    b, v0 = rng.standard_normal(csr.n), rng.standard_normal(csr.n)
    A = lib.Matrix(csr)
    P, _ = lib.Poly.build_ex(A, 8, dev(b), shift=9.0)
    r = lib.eigs(A, P, dev(v0), 30, 12, 6, rtol=1e-10, max_cycles=200)
    assert r.converged
    assert np.allclose(np.sort(r.mu.real), nearest(lam, 9.0, 6), rtol=0, atol=1e-8)


def _chain_bound(csr, mu, roots, growth, eps):
    nnzr = max(1.0, csr.nnz / csr.n) + 1
    amp = 1.0 + (O.infnorm(csr) + abs(mu)) / np.min(np.abs(roots))
    return (nnzr + 3) * len(roots) * eps * growth * amp


def test_shifted_apply_single_and_double(lib):
    """pi(A - mu I) v for a single polynomial with conjugate pairs, and for a
    double polynomial whose pi_1 ends with a conjugate pair and whose pi_2 has
    pairs: the last pass of that inner chain then combines five vectors and is
    split into a fused pass and a streaming combination."""
    csr = W.convdiff_2d(30, 1.6)
    mu = 0.35
    mv = shifted_mv(csr, mu)
    rng = np.random.default_rng(12)
    b, v = rng.standard_normal(csr.n), rng.standard_normal(csr.n)
    A = lib.Matrix(csr, want_f32=True)
    roots, _ = O.gmres_poly(mv, b, 14)
    assert np.any(roots.imag != 0)
    P = lib.Poly.from_roots(roots)
    P.shift = mu
    y = host(lib.apply(A, P, dev(v)))
    ref = O.apply_poly(mv, roots, v)
    g = max(np.abs(v).max(), np.abs(ref).max())
    w = v.copy()
    i = 0
    while i < len(roots):       # largest intermediate of the factored product
        st = 2 if roots[i].imag != 0 else 1
        w = O.apply_poly(mv, roots[i:i + st], w)
        g = max(g, np.abs(w).max())
        i += st
    assert np.max(np.abs(y - ref)) <= _chain_bound(csr, mu, roots, g, EPS64)
    # double polynomial with pairs at both levels and a pair last in pi_1
    r1, r2 = O.double_poly(mv, b, 4, 5)
    if r1[-1].imag == 0:
        cpx = [j for j in range(len(r1)) if r1[j].imag > 0]
        assert cpx, "need a conjugate pair in pi_1"
        j = cpx[0]
        order = [x for x in range(len(r1)) if x not in (j, j + 1)] + [j, j + 1]
        r1 = r1[order]
    assert r1[-1].imag != 0 and np.any(r2.imag != 0)
    D = lib.Poly.from_roots(r2, roots1=r1)
    D.shift = mu
    yd = host(lib.apply(A, D, dev(v)))
    refd = O.apply_double(mv, r1, r2, v)
    tau = lambda x: O.tau_apply(mv, r1, x)
    gd = np.abs(v).max()
    w = v.copy()
    i = 0
    while i < len(r2):
        st = 2 if r2[i].imag != 0 else 1
        w = O.apply_poly(tau, r2[i:i + st], w)
        gd = max(gd, np.abs(w).max())
        i += st
    tol = _chain_bound(csr, mu, r1, gd, EPS64) * len(r2) * 4
    assert np.max(np.abs(yd - refd)) <= tol
    y32 = host(lib.apply(A, D, dev(v, torch.float32), precision="f32")).astype(float)
    assert np.max(np.abs(y32 - refd)) <= tol * (EPS32 / EPS64) * 2
    # the byte count includes the extra streaming pass
    assert lib.apply_bytes(A, D, "f64") > 0
