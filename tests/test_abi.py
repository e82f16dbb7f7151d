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
        pytest.fail("libppa.so is not built (run python -m paper_1806_08020_amd.build)")
    import torch  # noqa: F401  (same HIP runtime as the product path)
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(cdll):
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(cdll, n)]
    assert not missing, missing


def test_bandwidth_probe_library_exports():
    """The benchmark's bandwidth reference kernels are built beside the
    solver library, as a library of their own."""
    path = os.path.join(ROOT, "paper_1806_08020_amd", "libppa_bwprobe.so")
    if not os.path.exists(path):
        pytest.fail("libppa_bwprobe.so is not built (run python -m paper_1806_08020_amd.build)")
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name in ("ppa_probe_read", "ppa_probe_read_wg", "ppa_probe_read_streams", "ppa_probe_copy",
                 "ppa_probe_read_write8", "ppa_probe_spmv_mix"):
        assert hasattr(lib, name), name


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


def test_host_dense_eig_several_triple_eigenvalues(cdll):
    """Non-normal matrices with several exactly triple eigenvalues (as a
    3-D operator with the same convection on every axis gives pi(A)): the
    shifted QR must reach the Schur form.  The first column of the
    double-shift product is formed from differences H(l, l) - shift; formed
    as H^2 - sH + tI it cancels to rounding noise once the shifts sit on a
    multiple eigenvalue, and the iteration then stalls (this family stalled
    in 74 of 200 draws)."""
    from paper_1806_08020_amd import ppa
    n = 40
    for seed in range(60):
        rng = np.random.default_rng([40, seed])
        k = 4 + 2 * (seed % 3)
        d = np.concatenate([np.repeat(rng.uniform(0.02, 0.3, k), 3), rng.uniform(-0.003, 0.01, n - 3 * k)])
        X = np.eye(n) + (0.1 + 0.1 * (seed % 3)) * rng.standard_normal((n, n))
        a = X @ np.diag(d) @ np.linalg.inv(X)
        w, V = ppa.dense_eig(a)
        # a triple eigenvalue perturbed at rounding level moves by about
        # cond(X) * eps * ||a||, first order (non-defective)
        tol = 1e-9 * np.linalg.cond(X)
        assert np.max(np.abs(np.sort(w.real) - np.sort(d))) <= tol, seed
        assert np.max(np.abs(w.imag)) <= tol
        R = a @ V - V * w
        assert np.linalg.norm(R) <= 1e-9 * np.linalg.norm(a) * n


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


def _ex7():
    from paper_1806_08020_amd import workloads as W
    lam = np.concatenate([np.arange(1, 100) / 10.0, np.arange(10, 9910), [20000.0]])
    return W.diag_csr(lam)


def test_host_stability_roots_match_oracle(cdll):
    """Section 7 on the host side of the library: log10 pof and the list with
    the extra copies placed equal the oracle's, element by element and in
    order, for Example 7's polynomials (d = 8, 25, 40), Example 9's outer
    polynomial, and hand-built lists with a conjugate pair and repeated roots."""
    import oracle as O
    from paper_1806_08020_amd import ppa
    A = _ex7()
    mv = O.csr_matvec(A)
    b = np.random.default_rng([7, 1]).standard_normal(A.n)
    cases = [O.gmres_poly(mv, b, d)[0] for d in (8, 25, 40)]
    b9 = np.random.default_rng(1).standard_normal(A.n)
    cases.append(O.double_poly(mv, b9, 5, 20)[1])
    z = 1e12 + 1e11j
    cases.append(np.array([z, np.conj(z), 2.0, 3.0, 4.0, 5.0], dtype=complex))
    cases.append(np.array([10.0, 2e10, 3.0, 4.0, 5.0], dtype=complex))
    cases.append(np.array([1.0, 1.0, 2.0], dtype=complex))     # repeated root: pof 0
    for roots in cases:
        P = ppa.Poly.from_roots(roots)
        lp = P.log10_pof()
        olp = O.log10_pof(roots)
        fin = np.isfinite(olp)
        assert np.array_equal(fin, np.isfinite(lp))
        assert np.allclose(lp[fin], olp[fin], rtol=0, atol=1e-11)
        S, added = P.stabilized()
        want, counts = O.add_stability_roots(roots)
        assert added == want.size - roots.size == int(np.sum(counts[roots.imag >= 0] *
                                                             np.where(roots[roots.imag >= 0].imag > 0, 2, 1)))
        assert S.degree == want.size
        assert np.array_equal(S.roots(), want)
    # a double polynomial keeps its other level untouched
    r1 = np.array([3.0, 7.0], dtype=complex)
    r2 = cases[3]
    D = ppa.Poly.from_roots(r2, roots1=r1)
    S2, added2 = D.stabilized(level=2)
    assert np.array_equal(S2.roots(1), r1) and added2 > 0
    assert np.array_equal(S2.roots(2), O.add_stability_roots(r2)[0])
    S1, added1 = D.stabilized(level=1)
    assert added1 == 0 and np.array_equal(S1.roots(2), r2)


def test_header_is_plain_c(tmp_path):
    """include/ppa.h compiles as C99 and as C++ on its own (no HIP or torch
    types in the boundary)."""
    import shutil
    import subprocess
    for compiler, std, ext in (("gcc", "-std=c99", "c"), ("g++", "-std=c++17", "cpp")):
        if shutil.which(compiler) is None:
            pytest.skip(f"{compiler} not available")
        src = tmp_path / f"use_header.{ext}"
        src.write_text('#include "ppa.h"\nint main(void) { return ppa_abi_version() == 1 ? 0 : 1; }\n')
        p = subprocess.run([compiler, std, "-Wall", "-Werror", "-fsyntax-only", "-I",
                            os.path.join(ROOT, "include"), str(src)], capture_output=True, text=True)
        assert p.returncode == 0, p.stderr
