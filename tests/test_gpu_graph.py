"""HIP-graph replay of the Krylov cycles (PPA_FLAG_GRAPH): each cycle's
operator applications and Gram-Schmidt launches are recorded once per start
column and basis buffer and replayed in later cycles.  The launches are the
same as in the eager run, so every result must be bitwise equal: values,
residuals, Ritz values and counters, after every number of cycles (each
replay follows the eager restart work and host synchronisation of the
previous cycle)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1806_08020_amd import workloads as W

from .test_gpu_parity import dev, host

pytestmark = pytest.mark.gpu


def _same(a, b):
    assert a.cycles == b.cycles and a.nconv == b.nconv
    assert np.array_equal(a.mu, b.mu) and np.array_equal(a.resid, b.resid)
    assert np.array_equal(a.nu, b.nu)
    assert (a.mvps, a.dots, a.vops, a.spmv_passes, a.spmv_passes_f32, a.spmv_bytes) == \
           (b.mvps, b.dots, b.vops, b.spmv_passes, b.spmv_passes_f32, b.spmv_bytes)


@pytest.mark.parametrize("kw", [dict(), dict(lowsync=True), dict(harmonic=True)])
def test_graph_replay_bitwise_every_cycle_count(lib, kw):
    """Convection-diffusion 40x40 (beta*h = 0.6), d = 3, Arnoldi(16,6): after
    1, 2, 3, 5 and 8 cycles the graph run equals the eager run bitwise."""
    csr = W.convdiff_2d(40, 0.6)
    b, v0 = W.start_vectors(csr.n, 3)
    A = lib.Matrix(csr)
    P = lib.Poly.build(A, 3, dev(b))
    for cycles in (1, 2, 3, 5, 8):
        g = lib.eigs(A, P, dev(v0), 16, 6, 6, rtol=0.0, max_cycles=cycles, graph=True, **kw)
        e = lib.eigs(A, P, dev(v0), 16, 6, 6, rtol=0.0, max_cycles=cycles, **kw)
        assert g.cycles == cycles
        _same(g, e)


def test_graph_mixed_precision_and_convergence(lib):
    """Mixed precision (the FP32-to-FP64 switch records a second set of
    graphs) on a 3-D convection-diffusion operator with a double polynomial,
    and a converging FP64 solve on the 50x50 Laplacian: bitwise equal to the
    eager runs; the Laplacian values are the closed-form ones."""
    csr = W.convdiff_3d(24, 0.3)
    b, v0 = W.start_vectors(csr.n, 5)
    A = lib.Matrix(csr, want_f32=True)
    P = lib.Poly.build_double(A, 4, 6, dev(b))
    g = lib.eigs(A, P, dev(v0), 30, 15, 8, rtol=1e-8, max_cycles=40, precision="mixed", graph=True)
    e = lib.eigs(A, P, dev(v0), 30, 15, 8, rtol=1e-8, max_cycles=40, precision="mixed")
    assert g.converged and g.fp32_cycles >= 1
    _same(g, e)
    csr = W.laplacian_2d(50)
    b, v0 = W.start_vectors(csr.n, 1)
    A = lib.Matrix(csr)
    P = lib.Poly.build(A, 10, dev(b))
    g = lib.eigs(A, P, dev(v0), 30, 15, 10, rtol=1e-8, max_cycles=100, graph=True)
    e = lib.eigs(A, P, dev(v0), 30, 15, 10, rtol=1e-8, max_cycles=100)
    assert g.converged and g.cycles > 2
    _same(g, e)
    i = np.arange(1, 51)
    lam = np.sort((4 - 2 * np.cos(i[:, None] * np.pi / 51) - 2 * np.cos(i[None, :] * np.pi / 51)).ravel())
    for mu in g.mu:
        assert np.min(np.abs(lam - mu.real)) <= 1e-10 * abs(mu.real)


def test_graph_solves_interleaved_with_eager_work(lib):
    """Graph solves on two matrices alternate with eager solves and plain
    fused passes on the same stream; every graph solve equals its eager twin."""
    mats = [W.convdiff_2d(40, 0.6), W.random_banded(20000, 27, 700, seed=4)]
    runs = []
    for csr in mats:
        b, v0 = W.start_vectors(csr.n, 6)
        A = lib.Matrix(csr)
        runs.append((A, lib.Poly.build(A, 5, dev(b)), dev(v0)))
    for rep in range(3):
        for A, P, v0 in runs:
            g = lib.eigs(A, P, v0, 20, 8, 6, rtol=0.0, max_cycles=4, graph=True)
            y = lib.fused_spmv(A, 1.0, v0, -0.5, v0)
            torch.cuda.synchronize()
            e = lib.eigs(A, P, v0, 20, 8, 6, rtol=0.0, max_cycles=4)
            _same(g, e)
            assert torch.isfinite(y).all()
