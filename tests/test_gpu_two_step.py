"""Two factors of pi per pass (ppa_matrix_two_step): for matrices of small
bandwidth a block computes two consecutive factors of eq. (2.1) in one
launch, the first on its rows widened by the bandwidth, kept in LDS.  The
products and row sums are those of the single passes, so pi(A)v, the
double polynomial and whole solves are bitwise the same with the form on
and off, in FP64 and FP32, with real roots, conjugate pairs and a shift;
pi(A)v also stays within the oracle's first-order bound.  Where the ranges
do not fit the LDS of a value type the form is refused for it."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1806_08020_amd import workloads as W

from .test_gpu_parity import EPS64, chain_tol, dev, host, oracle_chain

pytestmark = pytest.mark.gpu

CASES = {
    "convdiff2d_300": lambda: W.convdiff_2d(300, 0.5),       # bandwidth 300, conjugate pairs
    "laplacian_211": lambda: W.laplacian_2d(211),            # odd side, real roots only
    "band_60k": lambda: W.random_banded(60_000, 27, 300, seed=5),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_apply_bitwise_equal_to_single_passes(lib, name):
    csr = CASES[name]()
    A = lib.Matrix(csr, want_f32=True, two_step=True)
    on64, h = A.two_step("f64")
    on32, _ = A.two_step("f32")
    print(f"{name}: n={csr.n} bandwidth={h} on64={on64} on32={on32}", flush=True)
    assert on64 and on32 and h > 0
    b, v = W.start_vectors(csr.n, 3)
    P = lib.Poly.build(A, 12, dev(b))
    D = lib.Poly.build_double(A, 4, 5, dev(b))
    S = lib.Poly.from_roots(P.roots())
    S.shift = 0.25 * A.norm_inf          # pairs then carry the shift term
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        vt = dev(v, dt)
        for poly in (P, D, S):
            A.set_two_step(True, prec)
            y1 = lib.apply(A, poly, vt, precision=prec)
            A.set_two_step(False, prec)
            y0 = lib.apply(A, poly, vt, precision=prec)
            assert torch.isfinite(y1).all()
            assert torch.equal(y1, y0)
        A.set_two_step(True, prec)
    # the same algorithmic bytes are reported either way
    A.set_two_step(True)
    nb1 = lib.apply_bytes(A, P)
    A.set_two_step(False)
    assert lib.apply_bytes(A, P) == nb1


def test_apply_against_the_oracle(lib):
    """pi(A)v with the form on, FP64, against the oracle factor by factor."""
    csr = W.convdiff_2d(300, 1.2)
    mv = O.csr_matvec(csr)
    b, v = W.start_vectors(csr.n, 4)
    roots, _ = O.gmres_poly(mv, b, 14)
    assert np.any(roots.imag != 0) and np.any(roots.imag == 0)
    A = lib.Matrix(csr, two_step=True)
    assert A.two_step()[0]
    P = lib.Poly.from_roots(roots)
    y = host(lib.apply(A, P, dev(v)))
    ref, g = oracle_chain(mv, roots, v)
    assert np.max(np.abs(y - ref)) <= chain_tol(csr, roots, g, EPS64)


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_solve_bitwise_equal(lib, precision):
    """Whole solves (polynomial build, Arnoldi cycles on pi(A)) with the form
    on and off: the same pairs, residuals and counters."""
    csr = W.convdiff_2d(200, 0.4)
    b, v0 = W.start_vectors(csr.n, 6)
    out = {}
    for on in (True, False):
        A = lib.Matrix(csr, want_f32=True, two_step=True)
        A.set_two_step(on, "f64")
        A.set_two_step(on, "f32")
        P = lib.Poly.build(A, 15, dev(b))
        out[on] = lib.eigs(A, P, dev(v0), 30, 15, 8, rtol=1e-8, max_cycles=40, precision=precision)
    r1, r0 = out[True], out[False]
    assert r1.converged and r0.converged
    assert r1.cycles == r0.cycles and r1.spmv_passes == r0.spmv_passes
    assert np.array_equal(r1.mu, r0.mu) and np.array_equal(r1.resid, r0.resid)


@pytest.mark.parametrize("variant", ["graph", "harmonic", "lowsync"])
def test_solve_variants_with_the_form(lib, variant):
    """The solve's variants with two factors per pass: cycles replayed from
    HIP graphs, the harmonic restart and the delayed Gram-Schmidt each give
    the pairs of the same solve with the form off, bit for bit."""
    csr = W.convdiff_2d(180, 0.6)
    b, v0 = W.start_vectors(csr.n, 10)
    out = {}
    for on in (True, False):
        A = lib.Matrix(csr, two_step=True)
        A.set_two_step(on)
        P = lib.Poly.build(A, 12, dev(b))
        out[on] = lib.eigs(A, P, dev(v0), 30, 15, 8, rtol=1e-8, max_cycles=40, **{variant: True})
    r1, r0 = out[True], out[False]
    assert r1.converged and r0.converged and r1.cycles == r0.cycles
    assert np.array_equal(r1.mu, r0.mu) and np.array_equal(r1.resid, r0.resid)


def test_matrices_of_different_lds_needs_side_by_side(lib):
    """Two matrices whose ranges need different amounts of LDS, created in
    either order, both applied afterwards (the kernels' LDS limit is shared
    by all matrices)."""
    big = W.random_banded(60_000, 27, 900, seed=8)        # 80 KB of LDS, the small one 49 KB
    small = W.convdiff_2d(250, 0.5)
    for order in ((big, small), (small, big)):
        mats = [lib.Matrix(c, two_step=True) for c in order]
        for csr, A in zip(order, mats):
            assert A.two_step()[0]
            b, v = W.start_vectors(csr.n, 9)
            P = lib.Poly.build(A, 8, dev(b))
            y1 = lib.apply(A, P, dev(v))
            A.set_two_step(False)
            assert torch.equal(y1, lib.apply(A, P, dev(v)))
            A.set_two_step(True)


def test_refused_where_it_does_not_fit(lib):
    """Bandwidth 5000 at n = 60,000 (235 rows per block): the FP64 ranges do
    not fit 160 KB of LDS, the FP32 ones do; a row longer than 2048 nonzeros
    builds no records; the setter refuses what was not built."""
    csr = W.random_banded(60_000, 27, 5000, seed=6)
    A = lib.Matrix(csr, want_f32=True, two_step=True)
    on64, h = A.two_step("f64")
    on32, _ = A.two_step("f32")
    assert h >= 4900 and not on64 and on32
    with pytest.raises(lib.PPAError):
        A.set_two_step(True, "f64")
    b, v = W.start_vectors(csr.n, 7)
    P = lib.Poly.build(A, 8, dev(b))
    vt = dev(v, torch.float32)
    y1 = lib.apply(A, P, vt, precision="f32")
    A.set_two_step(False, "f32")
    assert torch.equal(y1, lib.apply(A, P, vt, precision="f32"))
    n = 5000
    Ad = np.eye(n) * 4.0
    Ad[np.arange(1, n), np.arange(n - 1)] = -1.0
    Ad[17, :2500] = 0.5                      # a row of 2500 nonzeros
    Al = lib.Matrix(W.dense_csr(Ad), two_step=True)
    assert Al.two_step() == (False, -1)
    with pytest.raises(lib.PPAError):
        Al.set_two_step(True)
    # without the flag nothing is built
    assert lib.Matrix(W.laplacian_2d(50)).two_step() == (False, -1)
