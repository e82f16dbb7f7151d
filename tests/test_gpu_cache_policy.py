"""Cache policies of the plain fused SpMV kernel (non-temporal or cached
matrix loads, plain or non-temporal output stores): they change how the
kernel uses the caches, never its arithmetic, so every policy's output is
bitwise the same, in FP64 and FP32, with and without the epilogue vectors,
including the mixed FP32-values / FP64-vector forms."""
import numpy as np
import pytest
import torch

from paper_1806_08020_amd import workloads as W

from .test_gpu_parity import EPS64, dev, host

pytestmark = pytest.mark.gpu

POL = ("stream", "keep", "keep_ntst")


@pytest.mark.parametrize("name", ["convdiff", "band", "long_rows"])
def test_policies_bitwise_equal(lib, name):
    if name == "convdiff":
        csr = W.convdiff_2d(300, 0.5)
    elif name == "band":
        csr = W.random_banded(50_000, 27, 700, seed=4)
    else:
        rng = np.random.default_rng(0)
        n = 6000
        A = np.zeros((n, n))
        A[np.arange(n), np.arange(n)] = 3.0
        A[7, :] = rng.standard_normal(n)        # a row longer than one block
        A[4000, ::2] = 1.0
        csr = W.dense_csr(A)
    A = lib.Matrix(csr, want_f32=True, window="off")
    rng = np.random.default_rng(5)
    u, x, z, z2 = (rng.standard_normal(csr.n) for _ in range(4))
    lens = np.diff(csr.rowptr)
    short = torch.as_tensor(lens <= 256, device="cuda")
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        outs = []
        for blocks in (2048, 256):
            A.set_spmv_blocks(blocks, prec)
            assert A.spmv_blocks(prec) == blocks
            for p in POL:
                A.set_cache_policy(p, prec)
                assert A.cache_policy(prec) == p
                outs.append((lib.fused_spmv(A, 0.5, dev(x, dt), -2.0, dev(u, dt)),
                             lib.fused_spmv(A, 0.5, dev(x, dt), -2.0, dev(u, dt), 1.5, dev(z, dt),
                                            -0.25, dev(z2, dt)),
                             lib.fused_spmv(A, 1.0, dev(u, dt), -0.5, dev(u, dt),
                                            out_dtype=torch.float64 if prec == "f32" else None)))
        # every policy of one block shape bitwise; the two shapes bitwise on
        # rows of at most 256 nonzeros and to rounding on longer ones
        for i in (1, 2, 4, 5):
            ref = outs[0] if i < 3 else outs[3]
            for a, b in zip(ref, outs[i]):
                assert torch.equal(a, b)
        for a, b in zip(outs[0], outs[3]):
            assert torch.equal(a[short], b[short])
            eps = 2.0 ** -52 if dt == torch.float64 else 2.0 ** -23
            assert torch.all((a - b).abs() <= 64 * eps * (a.abs() + b.abs() + 1))
        A.set_spmv_blocks(2048, prec)
    S = csr.to_scipy()
    ref = 0.5 * x - 2.0 * (S @ u) + 1.5 * z - 0.25 * z2
    nnzr = max(1, int(np.diff(csr.rowptr).max()))
    scale = 0.5 * np.abs(x) + 2 * (abs(S) @ np.abs(u)) + 1.5 * np.abs(z) + 0.25 * np.abs(z2)
    A.set_cache_policy("keep", "f64")
    y = host(lib.fused_spmv(A, 0.5, dev(x), -2.0, dev(u), 1.5, dev(z), -0.25, dev(z2)))
    assert np.all(np.abs(y - ref) <= (nnzr + 5) * EPS64 * scale)


def test_tuned_shape_c3_fp32_and_c2(lib):
    """The shape and policy the setup timing picked give the same bits as
    the defaults (large blocks, streaming loads) on the benchmark's 2-D
    operator and on a 3-D operator in FP32."""
    for csr, prec, dt in ((W.convdiff_2d(1000, 0.5), "f64", torch.float64),
                          (W.convdiff_3d(100, 0.3), "f32", torch.float32)):
        A = lib.Matrix(csr, want_f32=(prec == "f32"))
        assert A.spmv_blocks(prec) in (256, 2048)
        rng = np.random.default_rng(9)
        u = dev(rng.standard_normal(csr.n), dt)
        y1 = lib.fused_spmv(A, 1.0, u, -0.5, u)
        A.set_spmv_blocks(2048, prec)
        A.set_cache_policy("stream", prec)
        y0 = lib.fused_spmv(A, 1.0, u, -0.5, u)
        assert torch.equal(y0, y1)


def test_default_policy_and_errors(lib):
    """A matrix whose pass moves well under 128 MB keeps its stream cached by
    default; unknown policies and FP32 without FP32 values are rejected."""
    csr = W.laplacian_2d(50)
    A = lib.Matrix(csr)
    assert A.cache_policy("f64") == "keep"
    with pytest.raises(RuntimeError):
        A.set_cache_policy("keep", "f32")
    with pytest.raises(ValueError):
        A.set_cache_policy("bogus", "f64")
    assert A.spmv_blocks("f64") == 2048
    with pytest.raises(RuntimeError):
        A.set_spmv_blocks(1000, "f64")


def test_tuned_policy_full_size_bitwise(lib):
    """Convection-diffusion 1000x1000 (the benchmark's matrix): the policy the
    setup timing chose gives the same bits as the streaming policy."""
    csr = W.convdiff_2d(1000, 0.5)
    A = lib.Matrix(csr)
    chosen = A.cache_policy("f64")
    assert chosen in POL
    rng = np.random.default_rng(8)
    u, x = dev(rng.standard_normal(csr.n)), dev(rng.standard_normal(csr.n))
    y1 = lib.fused_spmv(A, 1.0, x, -0.5, u)
    A.set_cache_policy("stream", "f64")
    y0 = lib.fused_spmv(A, 1.0, x, -0.5, u)
    assert torch.equal(y0, y1)


def test_no_tune_keeps_size_rule(lib):
    """PPA_MATRIX_NO_TUNE: no timing at creation, so the size rule's cache
    policy and block shape (a pass served from the last-level cache with at
    least 1024 large blocks: the small blocks) and the plain kernel (a forced
    variant is still built); results equal the timed matrix's bit for bit.
    A smaller matrix keeps the large blocks."""
    small = lib.Matrix(W.convdiff_2d(400, 0.5), want_f32=True, tune=False)
    for prec in ("f64", "f32"):
        assert small.spmv_blocks(prec) == 2048
    csr = W.convdiff_2d(1000, 0.5)
    A = lib.Matrix(csr, want_f32=True, tune=False)
    for prec in ("f64", "f32"):
        assert A.spmv_blocks(prec) == 256
        assert A.cache_policy(prec) == "keep"
        assert A.spmv_variant(prec) == "plain"
    B = lib.Matrix(csr, want_f32=True)
    rng = np.random.default_rng(21)
    u = dev(rng.standard_normal(csr.n))
    assert torch.equal(lib.fused_spmv(A, 1.0, u, -0.5, u), lib.fused_spmv(B, 1.0, u, -0.5, u))
    R = lib.Matrix(W.random_banded(300_000, 9, 2000, seed=8), window="ring", tune=False)
    assert R.spmv_variant("f64") == "ring"
