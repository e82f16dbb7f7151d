"""GPU parity of the sliding-window SpMV (one persistent block per CU walks
consecutive row chunks and keeps u in an LDS ring).

It sums every row in column order like the plain kernel, so the two agree
bitwise on rows of at most 2048 nonzeros, in FP64, FP32 and the mixed
input/output forms, with and without the epilogue vectors; both are also
checked against the CSR product.  Matrices whose column ranges do not slide
(a far column, a band wider than the ring) are refused at setup and run on
another kernel.  Marked gpu; run on an MI355X."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1806_08020_amd import workloads as W

from .test_gpu_parity import EPS32, EPS64, chain_tol, dev, host, oracle_chain

pytestmark = pytest.mark.gpu


def ragged_band(n=150_000, band=3000, seed=7):
    """Band matrix with empty rows (every 97th, and a run of 700), rows of
    1 to 40 nonzeros and twelve rows of 600."""
    rng = np.random.default_rng([seed, 1])
    lens = rng.integers(1, 41, size=n)
    lens[::97] = 0
    lens[50_000:50_700] = 0
    lens[rng.choice(n, 12, replace=False)] = 600
    rows, cols = [], []
    for i in np.flatnonzero(lens):
        lo, hi = max(0, i - band), min(n, i + band + 1)
        c = rng.choice(np.arange(lo, hi), size=min(int(lens[i]), hi - lo), replace=False)
        rows.append(np.full(c.size, i))
        cols.append(c)
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    vals = rng.standard_normal(rows.size)
    return W._from_coo(n, rows, cols, vals)


def ring_mats():
    return {
        "band_200k": W.random_banded(200_000, 27, 5000, seed=5),
        "ragged": ragged_band(),
        "cd2_600": W.convdiff_2d(600, 0.5),
        "band_9000": W.random_banded(9000, 27, 700, seed=4),
        "lap_50": W.laplacian_2d(50),
        "diag_5000": W.diag_csr(np.linspace(0.1, 9.0, 5000)),
    }


MATS = ring_mats()


@pytest.mark.parametrize("name", list(MATS))
def test_ring_bitwise_equal_to_plain(lib, name):
    csr = MATS[name]
    Ar = lib.Matrix(csr, want_f32=True, window="ring")
    Ap = lib.Matrix(csr, want_f32=True, window="off")
    assert Ar.spmv_variant("f64") == "ring" and Ar.spmv_variant("f32") == "ring"
    assert Ap.spmv_variant("f64") == "plain" and Ap.spmv_variant("f32") == "plain"
    rng = np.random.default_rng(11)
    u, x, z, z2 = (rng.standard_normal(csr.n) for _ in range(4))
    for in_t, out_t in ((torch.float64, torch.float64), (torch.float32, torch.float32),
                        (torch.float64, torch.float32), (torch.float32, torch.float64)):
        args = (0.5, dev(x, in_t), -2.0, dev(u, in_t), 1.5, dev(z, in_t), -0.25, dev(z2, in_t))
        yr = lib.fused_spmv(Ar, *args, out_dtype=out_t)
        yp = lib.fused_spmv(Ap, *args, out_dtype=out_t)
        assert torch.equal(yr, yp), (in_t, out_t)
        yr = lib.fused_spmv(Ar, 1.0, dev(x, in_t), -0.4, dev(u, in_t), out_dtype=out_t)
        yp = lib.fused_spmv(Ap, 1.0, dev(x, in_t), -0.4, dev(u, in_t), out_dtype=out_t)
        assert torch.equal(yr, yp), (in_t, out_t)
    S = csr.to_scipy()
    ref = 0.5 * x - 2.0 * (S @ u) + 1.5 * z - 0.25 * z2
    scale = 0.5 * np.abs(x) + 2 * (abs(S) @ np.abs(u)) + 1.5 * np.abs(z) + 0.25 * np.abs(z2)
    nnzr = max(1, int(np.diff(csr.rowptr).max()))
    y = host(lib.fused_spmv(Ar, 0.5, dev(x), -2.0, dev(u), 1.5, dev(z), -0.25, dev(z2)))
    assert np.all(np.abs(y - ref) <= (nnzr + 4) * EPS64 * scale + 1e-300)
    y32 = host(lib.fused_spmv(Ar, 0.5, dev(x, torch.float32), -2.0, dev(u, torch.float32), 1.5,
                              dev(z, torch.float32), -0.25, dev(z2, torch.float32))).astype(float)
    assert np.all(np.abs(y32 - ref) <= (nnzr + 6) * 2 * EPS32 * scale + 1e-30)


def test_ring_repeated_calls_and_aliasing_rules(lib):
    """Repeated passes give the same bits; out must not alias u."""
    csr = MATS["band_200k"]
    A = lib.Matrix(csr, window="ring")
    rng = np.random.default_rng(12)
    u, x = dev(rng.standard_normal(csr.n)), dev(rng.standard_normal(csr.n))
    y1 = lib.fused_spmv(A, 1.0, x, 0.3, u)
    y2 = lib.fused_spmv(A, 1.0, x, 0.3, u)
    assert torch.equal(y1, y2)
    with pytest.raises(lib.PPAError):
        lib.fused_spmv(A, 1.0, x, 0.3, u, out=u)


def test_ring_refused_when_columns_do_not_slide(lib):
    """A far column in the first row makes the first segment's column range
    wider than the ring; a band of +-9000 exceeds the FP64 ring (12288
    entries) but fits the FP32 one (24576)."""
    base = W.random_banded(300_000, 9, 2000, seed=8)
    coo = base.to_scipy().tocoo()
    keep = ~((coo.row == 0) & (coo.col == base.n - 1))
    far = W._from_coo(base.n, np.append(coo.row[keep], 0), np.append(coo.col[keep], base.n - 1),
                      np.append(coo.data[keep], 1.0))
    A = lib.Matrix(far, want_f32=True, window="ring")
    assert A.spmv_variant("f64") != "ring" and A.spmv_variant("f32") != "ring"
    wide = W.random_banded(100_000, 9, 9000, seed=9)
    B = lib.Matrix(wide, want_f32=True, window="ring")
    assert B.spmv_variant("f64") != "ring"
    assert B.spmv_variant("f32") == "ring"
    rng = np.random.default_rng(13)
    u = rng.standard_normal(wide.n)
    Bp = lib.Matrix(wide, want_f32=True, window="off")
    for A_, t in ((B, torch.float64), (B, torch.float32)):
        assert torch.equal(lib.fused_spmv(A_, 0.0, None, 1.0, dev(u, t)),
                           lib.fused_spmv(Bp, 0.0, None, 1.0, dev(u, t)))


def test_ring_apply_matches_oracle(lib):
    csr = MATS["band_200k"]
    mv = O.csr_matvec(csr)
    b, v = W.start_vectors(csr.n, 14)
    roots, _ = O.gmres_poly(mv, b, 12)
    A = lib.Matrix(csr, want_f32=True, window="ring")
    P = lib.Poly.from_roots(roots)
    y = host(lib.apply(A, P, dev(v)))
    ref, g = oracle_chain(mv, roots, v)
    assert np.max(np.abs(y - ref)) <= chain_tol(csr, roots, g, EPS64)
    y32 = host(lib.apply(A, P, dev(v, torch.float32), precision="f32")).astype(float)
    assert np.max(np.abs(y32 - ref)) <= chain_tol(csr, roots, g, EPS64) * (EPS32 / EPS64) * 2


def test_ring_eigs_identical_to_plain(lib):
    """Every SpMV agrees bitwise, so whole restart cycles do too."""
    csr = MATS["cd2_600"]
    b, v0 = W.start_vectors(csr.n, 15)
    out = []
    for window in ("ring", "off"):
        A = lib.Matrix(csr, want_f32=True, window=window)
        P = lib.Poly.build(A, 15, dev(b))
        r = lib.eigs(A, P, dev(v0), 30, 12, 5, rtol=1e-8, max_cycles=2, precision="mixed")
        out.append((P.roots(), r.mu, r.resid, r.cycles, r.mvps))
    (ra, ma, sa, ca, va), (rb, mb, sb, cb, vb) = out
    assert np.array_equal(ra, rb)
    assert np.array_equal(ma, mb) and np.array_equal(sa, sb)
    assert ca == cb and va == vb


def test_ring_unaligned_values_take_the_narrow_loads(lib):
    """FP64 values whose array is 8- but not 16-byte aligned cannot be read
    two nonzeros per 16-byte load: the sliding-window kernel then loads them
    one per lane, with the same bits as the plain kernel and as the aligned
    handle."""
    import ctypes
    from paper_1806_08020_amd import ppa
    csr = MATS["band_200k"]
    Aa = lib.Matrix(csr, window="ring")
    Ap = lib.Matrix(csr, window="off")
    buf = torch.empty(csr.nnz + 1, dtype=torch.float64, device="cuda")
    buf[1:] = Aa.vals
    vals = buf[1:]
    assert vals.data_ptr() % 16 == 8
    Au = object.__new__(ppa.Matrix)
    Au.n, Au.rowptr, Au.colind, Au.vals, Au.vals32 = csr.n, Aa.rowptr, Aa.colind, vals, None
    h = ctypes.c_void_p()
    ppa._check(ppa._lib.ppa_matrix_create(csr.n, ppa._ptr(Aa.rowptr), ppa._ptr(Aa.colind), ppa._ptr(vals),
                                          None, ppa.PPA_MATRIX_RING_FORCE, ppa._stream(), ctypes.byref(h)))
    Au.h = h
    Au.nnz, Au.norm_inf, Au.nblocks = Aa.nnz, Aa.norm_inf, Aa.nblocks
    Au._keep = buf
    assert Au.spmv_variant("f64") == "ring"
    rng = np.random.default_rng(17)
    u, x, z = (dev(rng.standard_normal(csr.n)) for _ in range(3))
    for args in ((0.5, x, -2.0, u), (1.0, u, -0.25, u), (0.5, x, -2.0, u, 1.5, z)):
        yu = lib.fused_spmv(Au, *args)
        assert torch.equal(yu, lib.fused_spmv(Aa, *args))
        assert torch.equal(yu, lib.fused_spmv(Ap, *args))
