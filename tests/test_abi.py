"""The C-ABI library loads on the CPU, exports every entry point declared in
include/ppa.h, and its host-only routines (small dense eigensolver, Leja
ordering) agree with NumPy / the oracle.  No device compute here."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "ppa.h")
LIB = os.path.join(ROOT, "paper_1806_08020_amd", "libppa.so")


def declared_functions():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ppa_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def cdll():
    if not os.path.exists(LIB):
        pytest.fail("libppa.so is not built (run __graft_entry__.build())")
    import torch  # noqa: F401  (same HIP runtime as the product path)
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(cdll):
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(cdll, n)]
    assert not missing, missing


def test_abi_version(cdll):
    from paper_1806_08020_amd import ppa
    assert ppa.abi_version() == 1


@pytest.mark.parametrize("seed,n", [(0, 1), (1, 2), (2, 7), (3, 30), (4, 64), (5, 120)])
def test_host_dense_eig_matches_numpy(cdll, seed, n):
    from paper_1806_08020_amd import ppa
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n))
    w, V = ppa.dense_eig(a)
    ref = np.linalg.eigvals(a)
    for z in ref:
        assert np.min(np.abs(w - z)) <= 1e-9 * max(1.0, np.abs(ref).max())
    # conjugate pairs adjacent, Im > 0 first
    i = 0
    while i < n:
        if w[i].imag != 0:
            assert w[i].imag > 0 and w[i + 1] == np.conj(w[i])
            i += 2
        else:
            i += 1
    # eigenvectors: A v = w v, unit norm
    R = a @ V - V * w
    assert np.linalg.norm(R) <= 1e-9 * np.linalg.norm(a) * n
    assert np.allclose(np.linalg.norm(V, axis=0), 1.0)


def test_host_dense_eig_symmetric_and_repeated(cdll):
    from paper_1806_08020_amd import ppa
    rng = np.random.default_rng(9)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    lam = np.array([1, 1, 2, 3, 3, 3, 4, 5, 6, 7, 8, 9.0])
    a = Q @ np.diag(lam) @ Q.T
    w = ppa.dense_eig(a, vectors=False)
    assert np.allclose(np.sort(w.real), lam, atol=1e-12)
    # Hessenberg with exact zero subdiagonal, and a rotation block
    b = np.zeros((4, 4)); b[0, 0] = 2; b[1:3, 1:3] = [[0, -1], [1, 0]]; b[3, 3] = -5
    wb = ppa.dense_eig(b, vectors=False)
    assert sorted(map(lambda z: (round(z.real, 12), round(z.imag, 12)), wb)) == \
        sorted([(2, 0), (0, 1), (0, -1), (-5, 0)])


@pytest.mark.parametrize("seed", range(6))
def test_host_leja_matches_oracle(cdll, seed):
    import oracle as O
    from paper_1806_08020_amd import ppa
    rng = np.random.default_rng(50 + seed)
    th = list(rng.uniform(-2, 9, 9))
    for _ in range(4):
        z = complex(rng.uniform(0, 6), rng.uniform(0.05, 3))
        th += [z, np.conj(z)]
    th += [th[0], th[9], np.conj(th[9])]      # repeated roots go last
    th = np.array(th, dtype=complex)
    rng.shuffle(th)
    assert np.array_equal(ppa.leja_order(th), O.leja_order(th))


def test_host_eigvecs_accurate_on_restarted_arnoldi(cdll):
    """After a thick restart H_m is nearly block triangular (tiny spike row);
    the host eigenvectors must stay accurate in norm, which the restart basis
    and the Ritz test rely on."""
    import oracle as O
    from paper_1806_08020_amd import ppa
    from paper_1806_08020_amd import workloads as W
    csr = W.convdiff_2d(36, 0.6)
    b, v0 = W.start_vectors(csr.n, 21)
    mats = []
    O.pp_eigs(csr, b, v0, m=38, k=19, nev=14, d=27, rtol=1e-12, max_cycles=6,
              hook=lambda ev, V, H, j: mats.append(H[:j, :j].copy()) if ev == "cycle" else None)
    assert len(mats) >= 3
    for Hm in mats:
        w, V = ppa.dense_eig(Hm)
        R = Hm @ V - V * w
        assert np.linalg.norm(R, axis=0).max() <= 1e-13 * np.linalg.norm(Hm)
