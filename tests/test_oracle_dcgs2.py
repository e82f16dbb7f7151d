"""Pins of the oracle's delayed-reorthogonalisation Arnoldi
(``arnoldi_extend_dcgs2``: one block of inner products per step, the second
Gram-Schmidt pass of step j-1 merged with the first pass of step j).  It
must build the same Arnoldi decomposition as Gram-Schmidt with an immediate
reorthogonalisation pass (exact arithmetic gives identical V and H), with an
orthonormal basis and the Arnoldi relation to rounding."""
import inspect
import textwrap

import numpy as np
import pytest

import oracle as O
import oracle.ppa_oracle as P
from paper_1806_08020_amd import workloads as W


def _cgs2_extend(op, V, H, j0, m):
    for j in range(j0, m):
        w = op(V[:, j])
        w0 = np.linalg.norm(w)
        h, w, beta = O.cgs2(V[:, : j + 1], w)
        H[: j + 1, j] = h
        if beta <= O.BREAKDOWN_TOL * w0:
            H[j + 1, j] = 0.0
            return j + 1, True
        H[j + 1, j] = beta
        V[:, j + 1] = w / beta
    return m, False


def _operators():
    cd = W.convdiff_2d(30, 0.5)
    mv = O.csr_matvec(cd)
    b, _ = W.start_vectors(cd.n, 3)
    roots, _ = O.gmres_poly(mv, b, 8)
    rng = np.random.default_rng(11)
    D = rng.standard_normal((300, 300)) / np.sqrt(300) + np.diag(np.linspace(1, 4, 300))
    g = np.geomspace(1e-12, 1.0, 400)
    return {"convdiff_poly": (cd.n, lambda x: O.apply_poly(mv, roots, x)),
            "dense_nonsym": (300, lambda x: D @ x),
            "graded_diag": (400, lambda x: g * x)}


def _extend(fn, n, op, m, seed, j0=0, V=None, H=None):
    if V is None:
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        V[:, 0] = np.random.default_rng(seed).standard_normal(n)
        V[:, 0] /= np.linalg.norm(V[:, 0])
    mc, broke = fn(op, V, H, j0, m)
    return V, H, mc, broke


@pytest.mark.parametrize("name", ["convdiff_poly", "dense_nonsym", "graded_diag"])
def test_matches_immediate_reorthogonalisation(name, fn=None):
    """Same start vector: V and H equal those of the immediate form to
    rounding; V orthonormal; op V_m = V_{m+1} Hbar.  The graded diagonal
    (eigenvalues 1e-12..1, geometric) drives the subdiagonal of H far below
    its norm, where the terms that correct for the lagged pass matter; the
    bounds there are a few times the clean run's (orthonormality 6.7e-16,
    relation 1.3e-16)."""
    fn = fn or O.arnoldi_extend_dcgs2
    n, op = _operators()[name]
    m = 40 if name == "graded_diag" else 30
    V1, H1, mc1, _ = _extend(_cgs2_extend, n, op, m, 5)
    V2, H2, mc2, _ = _extend(fn, n, op, m, 5)
    assert mc1 == mc2 == m
    assert np.abs(V2.T @ V2 - np.eye(m + 1)).max() <= 2e-15
    R = np.column_stack([op(V2[:, j]) for j in range(m)]) - V2 @ H2
    assert np.linalg.norm(R) <= 4e-16 * np.linalg.norm(H2)
    assert np.abs(H2 - H1).max() <= 1e-11 * np.abs(H1).max()
    assert np.abs(V2 - V1).max() <= 1e-11


def test_continues_a_restarted_basis():
    """Started at j0 > 0 from a Krylov-like decomposition with a full block
    (as a thick restart leaves it), the extension keeps the relation and
    orthonormality."""
    n, op = _operators()["convdiff_poly"]
    m, kk = 30, 9
    V, H, _, _ = _extend(_cgs2_extend, n, op, m, 7)
    # rotate the first m vectors: V_kk = V_m Q, v_{kk+1} = v_{m+1}
    Hm = H[:m, :m]
    _, Z = np.linalg.eig(Hm)
    Q, _ = np.linalg.qr(np.real(Z[:, :kk]) + 0.3 * np.imag(Z[:, :kk]))
    Vn = np.zeros_like(V)
    Hn = np.zeros_like(H)
    Vn[:, :kk] = V[:, :m] @ Q
    Vn[:, kk] = V[:, m]
    Hn[:kk, :kk] = Q.T @ Hm @ Q
    Hn[kk, :kk] = H[m, m - 1] * Q[m - 1, :]
    Vn2, Hn2 = Vn.copy(), Hn.copy()
    O.arnoldi_extend_dcgs2(op, Vn, Hn, kk, m)
    assert np.abs(Vn.T @ Vn - np.eye(m + 1)).max() <= 1e-13
    R = np.column_stack([op(Vn[:, j]) for j in range(m)]) - Vn @ Hn
    assert np.linalg.norm(R) <= 1e-13 * np.linalg.norm(Hn)
    _cgs2_extend(op, Vn2, Hn2, kk, m)
    assert np.abs(Hn - Hn2).max() <= 1e-10 * np.abs(Hn2).max()


def test_breakdown_on_invariant_subspace():
    """A = diag with five distinct values: the Krylov space is invariant after
    five steps; both forms stop there with the same H."""
    d = np.repeat([1.0, 2.0, 3.5, 5.0, 8.0], 40)
    op = lambda x: d * x
    V1, H1, mc1, b1 = _extend(_cgs2_extend, d.size, op, 12, 2)
    V2, H2, mc2, b2 = _extend(O.arnoldi_extend_dcgs2, d.size, op, 12, 2)
    assert b1 and b2 and mc1 == mc2 == 5
    assert np.allclose(H1[:6, :5], H2[:6, :5], rtol=0, atol=1e-12)
    assert np.allclose(np.sort(np.linalg.eigvals(H2[:5, :5]).real), [1, 2, 3.5, 5, 8], atol=1e-12)


@pytest.mark.parametrize("N,bh,nev", [(50, 0.0, 10), (20, 0.5, 6)])
def test_solve_closed_form(N, bh, nev):
    """Polynomial preconditioned Arnoldi with the delayed form reaches the
    closed-form smallest eigenvalues (Laplacian 50x50, convection-diffusion
    20x20 with beta*h = 0.5), with the same cycle count as the immediate form."""
    A = W.laplacian_2d(N) if bh == 0.0 else W.convdiff_2d(N, bh)
    g = bh / 2
    i = np.arange(1, N + 1)
    lam = np.sort((4 - 2 * np.sqrt(1 - g * g) * np.cos(i[:, None] * np.pi / (N + 1))
                   - 2 * np.cos(i[None, :] * np.pi / (N + 1))).ravel())
    rng = np.random.default_rng([N, 2])
    b, v0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    kw = dict(d=10 if bh == 0 else 8, rtol=1e-10, max_cycles=200)
    r2, _ = O.pp_eigs(A, b, v0, 30, 15, nev, ortho="dcgs2", **kw)
    r1, _ = O.pp_eigs(A, b, v0, 30, 15, nev, **kw)
    assert r2.converged and abs(r2.cycles - r1.cycles) <= 1
    assert np.allclose(np.sort(r2.mu.real), lam[:nev], rtol=0, atol=1e-8)


# ---------------------------------------------------------------- planted mistakes
def _mutant(old, new):
    src = textwrap.dedent(inspect.getsource(P.arnoldi_extend_dcgs2))
    assert old in src
    ns = dict(P.__dict__)
    exec(src.replace(old, new, 1), ns)
    return ns["arnoldi_extend_dcgs2"]


# a, c and a^T b vanish in exact arithmetic (u is orthogonal to Q there):
# dropping one of them (the H correction, a^T a in beta, a^T b or c[j] in
# h[j]) changes V and H by rounding only, at most 2e-15 relative on these
# operators, which no FP64 pin separates.  The terms below change results
# beyond rounding.
@pytest.mark.parametrize("old,new", [
    ("gamma = (c[j] / beta + hj) / beta", "gamma = hj / beta"),      # q_j's coefficient
    ("htop = (b - c[:j]) / beta", "htop = b / beta"),                # op(Q) a dropped
    ("g = c[:j] / beta + htop - gamma * a", "g = htop - gamma * a"),
    ("g = c[:j] / beta + htop - gamma * a", "g = c[:j] / beta + htop"),
    ("V[:, j] = (u - Q @ a) / beta", "V[:, j] = u / beta"),          # second pass not applied
    ("u = w / beta - gamma * u - Q @ g", "u = w / beta - gamma * u + Q @ g"),
])
def test_mutant_is_caught(old, new):
    fn = _mutant(old, new)
    with pytest.raises(AssertionError):
        for name in ("convdiff_poly", "dense_nonsym", "graded_diag"):
            test_matches_immediate_reorthogonalisation(name, fn=fn)
