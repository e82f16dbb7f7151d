"""The allocation-free apply (static per-device scratch) against the
workspace apply: same kernels, so the outputs must agree bit for bit.  Two
calls in a row, the second on a smaller problem; FP32 too; a request larger
than the static array is refused on the host and leaves the output alone."""
import numpy as np
import pytest
import torch

from paper_1806_08020_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(lib, csr, d, seed, double=False, f32=False):
    A = lib.Matrix(csr, want_f32=f32)
    b, v = W.start_vectors(csr.n, seed)
    bt = torch.as_tensor(b, device="cuda")
    P = lib.Poly.build_double(A, d[0], d[1], bt) if double else lib.Poly.build(A, d, bt)
    dt = torch.float32 if f32 else torch.float64
    vt = torch.as_tensor(v, device="cuda").to(dt)
    return A, P, vt


def _check_pair(lib, A, P, vt, precision):
    ref = lib.apply(A, P, vt, precision=precision)
    y = torch.full_like(vt, float("nan"))
    lib.apply_noalloc(A, P, vt, precision=precision, out=y)
    torch.cuda.synchronize()
    print(f"noalloc n={A.n} degree={P.roots().size} {precision}", flush=True)
    assert torch.isfinite(ref).all()
    assert torch.equal(y, ref)


def test_two_calls_second_smaller(lib):
    # first: 2-D convection-diffusion 300x300, degree 20 (four n-vectors of scratch)
    A1, P1, v1 = _case(lib, W.convdiff_2d(300, 0.5), 20, 11)
    _check_pair(lib, A1, P1, v1, "f64")
    # second, smaller: a double polynomial (six n-vectors) on a 40x41 Laplacian
    A2, P2, v2 = _case(lib, W.laplacian_2d(40, 41), (3, 4), 12, double=True)
    _check_pair(lib, A2, P2, v2, "f64")
    # the scratch keeps the first call's contents: run the large one again
    _check_pair(lib, A1, P1, v1, "f64")


def test_fp32_chain(lib):
    A, P, v = _case(lib, W.convdiff_2d(120, 0.3), 12, 13, f32=True)
    _check_pair(lib, A, P, v, "f32")
    A2, P2, v2 = _case(lib, W.convdiff_2d(50, 0.3), (2, 3), 14, double=True, f32=True)
    _check_pair(lib, A2, P2, v2, "f32")


def test_request_beyond_the_array_is_refused(lib):
    # FP64 single polynomial: 4 n-vectors; n = 2.2e6 needs 70.4 MB > 64 MiB
    n = 2_200_000
    csr = W.diag_csr(np.linspace(1.0, 2.0, n))
    A = lib.Matrix(csr, tune=False)
    P = lib.Poly.from_roots(np.array([1.5, 3.0]))
    v = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.full_like(v, -7.0)
    with pytest.raises(lib.PPAError) as e:
        lib.apply_noalloc(A, P, v, out=y)
    assert e.value.status == lib.PPA_ERR_WORKSPACE
    assert "static array" in str(e.value)
    torch.cuda.synchronize()
    assert bool((y == -7.0).all())
    # the same request fits the workspace entry point, and a smaller one the array
    ref = lib.apply(A, P, v)
    lam = torch.as_tensor(csr.vals, device="cuda")
    assert torch.allclose(ref, (1 - lam / 1.5) * (1 - lam / 3.0), rtol=0, atol=1e-15)
    A2, P2, v2 = _case(lib, W.laplacian_2d(30), 6, 15)
    _check_pair(lib, A2, P2, v2, "f64")
