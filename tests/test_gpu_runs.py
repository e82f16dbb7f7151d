"""Column runs of the plain fused SpMV kernel: a block copies the contiguous
runs of u its rows gather from into LDS and reads its gathers there.  The
products and row sums are unchanged, so the output is bitwise that of the
same kernel gathering from memory, in FP64, FP32 and the mixed
FP32-values / FP64-vector forms, with and without the epilogue vectors;
blocks whose runs do not fit (too many, too long, a long row) gather from
memory inside the same launch; when x is the gathered vector itself its
entries come from the runs too (they cover the block's rows); a gathered
vector that is not 16-byte aligned sends the launch to the plain form."""
import numpy as np
import pytest
import torch

from paper_1806_08020_amd import workloads as W

from .test_gpu_parity import dev

pytestmark = pytest.mark.gpu


def _with_far_entries(csr, every, seed):
    """csr plus one entry at a random far column in every `every`-th row
    (columns stay sorted and distinct): those blocks get extra runs."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(csr.n):
        c = csr.colind[csr.rowptr[i]:csr.rowptr[i + 1]].tolist()
        v = csr.vals[csr.rowptr[i]:csr.rowptr[i + 1]].tolist()
        if i % every == 0:
            f = int(rng.integers(0, csr.n))
            if f not in c:
                c.append(f)
                v.append(0.125)
        o = np.argsort(c)
        rows.append((np.asarray(c)[o], np.asarray(v)[o]))
    rp = np.zeros(csr.n + 1, np.int64)
    rp[1:] = np.cumsum([len(r[0]) for r in rows])
    return W.CSR(csr.n, rp.astype(np.int32), np.concatenate([r[0] for r in rows]).astype(np.int32),
                 np.concatenate([r[1] for r in rows]))


def _long_rows(n, seed):
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n))
    A[np.arange(n), np.arange(n)] = 3.0
    A[np.arange(1, n), np.arange(n - 1)] = -1.0
    A[11, :] = rng.standard_normal(n)        # longer than one block
    A[n // 2, ::3] = 1.0
    A[n - 1, :] = 0.0                        # an empty last row
    A[n // 3, :] = 0.0                       # and an empty interior one
    return W.dense_csr(A)


CASES = {
    "convdiff3d_odd": lambda: W.convdiff_3d(37, 0.2),           # n = 50653, odd
    "convdiff3d": lambda: W.convdiff_3d(48, 0.3),
    "convdiff2d": lambda: W.convdiff_2d(400, 0.5),
    "far_entries": lambda: _with_far_entries(W.convdiff_3d(30, 0.3), 40, 3),
    "band_wide": lambda: W.random_banded(60_000, 27, 5000, seed=4),   # runs too long: memory gathers
    "long_rows": lambda: _long_rows(6000, 1),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_runs_bitwise_equal_to_memory_gathers(lib, name):
    csr = CASES[name]()
    A = lib.Matrix(csr, want_f32=True, window="runs")
    rng = np.random.default_rng(7)
    u, x, z, z2 = (rng.standard_normal(csr.n) for _ in range(4))
    with_runs = {p: A.spmv_runs(p) for p in ("f64", "f32")}
    print(f"{name}: n={csr.n} nnz={csr.nnz} blocks={A.nblocks} runs={with_runs}", flush=True)
    if name in ("convdiff3d", "convdiff3d_odd", "convdiff2d", "far_entries"):
        for p in ("f64", "f32"):
            assert with_runs[p][0] and with_runs[p][1] > 0
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        outs = {}
        for on in (True, False):
            if with_runs[prec][0] or not on:
                A.set_spmv_runs(on, prec)
            assert A.spmv_runs(prec)[0] == (on and with_runs[prec][0])
            assert A.spmv_blocks(prec) == 2048
            ut = dev(u, dt)
            o = [lib.fused_spmv(A, 0.5, dev(x, dt), -2.0, dev(u, dt)),
                 lib.fused_spmv(A, 1.0, ut, -0.5, ut),          # x is u: x read from the runs
                 lib.fused_spmv(A, 0.5, dev(x, dt), -2.0, dev(u, dt), 1.5, dev(z, dt), -0.25, dev(z2, dt)),
                 lib.fused_spmv(A, 1.0, dev(u, dt), -0.5, dev(u, dt))]
            if prec == "f32":
                # FP32 values with FP64 vectors in, FP32 out (and the reverse)
                o.append(lib.fused_spmv(A, 1.0, dev(u, torch.float64), -0.5, dev(u, torch.float64),
                                        out_dtype=torch.float32))
                o.append(lib.fused_spmv(A, 1.0, dev(u, dt), -0.5, dev(u, dt), out_dtype=torch.float64))
            outs[on] = o
        for a, b in zip(outs[True], outs[False]):
            assert torch.isfinite(a).all()
            assert torch.equal(a, b)


def test_unaligned_gathered_vector(lib):
    csr = W.convdiff_3d(30, 0.3)
    A = lib.Matrix(csr, window="runs")
    assert A.spmv_runs("f64")[0]
    buf = torch.as_tensor(np.random.default_rng(2).standard_normal(csr.n + 1), device="cuda")
    u = buf[1:]                      # 8-byte aligned only
    y1 = lib.fused_spmv(A, 1.0, u, -0.5, u)
    A.set_spmv_runs(False)
    y0 = lib.fused_spmv(A, 1.0, u, -0.5, u)
    assert torch.equal(y1, y0)


def test_apply_chain_with_runs(lib):
    # a whole double-polynomial application: runs on and off agree bitwise
    csr = W.convdiff_3d(40, 0.3)
    A = lib.Matrix(csr, want_f32=True, window="runs")
    b, v = W.start_vectors(csr.n, 21)
    P = lib.Poly.build_double(A, 4, 5, torch.as_tensor(b, device="cuda"))
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        vt = torch.as_tensor(v, device="cuda").to(dt)
        A.set_spmv_runs(True, prec)
        y1 = lib.apply(A, P, vt, precision=prec)
        A.set_spmv_runs(False, prec)
        y0 = lib.apply(A, P, vt, precision=prec)
        assert torch.equal(y1, y0)


def test_runs_setter_needs_built_runs(lib):
    A = lib.Matrix(W.convdiff_2d(50, 0.5), window="off")
    assert A.spmv_runs("f64") == (False, 0)
    with pytest.raises(lib.PPAError):
        A.set_spmv_runs(True)
    A.set_spmv_runs(False)
