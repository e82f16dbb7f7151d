"""Pins of the oracle's stability control (section 7, 'Adding roots for
stability', and its use on a double polynomial in section 8, Example 9)
against the mathematics and the paper's printed results."""
import os

import mpmath
import numpy as np
import pytest

import oracle as O
from paper_1806_08020_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def ex7_matrix():
    lam = np.concatenate([np.arange(1, 100) / 10.0, np.arange(10, 9910), [20000.0]])
    assert lam.size == 10000
    return W.diag_csr(lam)


def test_pof_is_scaled_derivative():
    """|pi'(theta_j)| = pof(j) / |theta_j| for pi(z) = prod (1 - z/theta_i):
    the derivative taken numerically in 40-digit arithmetic."""
    rng = np.random.default_rng(3)
    re = rng.uniform(0.5, 5.0, 5)
    theta = np.concatenate([re, [2.0 + 1.5j, 2.0 - 1.5j]])
    mpmath.mp.dps = 40
    th = [mpmath.mpc(z.real, z.imag) for z in theta]

    def pi(z):
        p = mpmath.mpf(1)
        for t in th:
            p *= (1 - z / t)
        return p

    p = O.pof(theta)
    for j, t in enumerate(th):
        dp = mpmath.diff(pi, t)
        assert abs(float(abs(dp)) - p[j] / abs(theta[j])) <= 1e-12 * p[j] / abs(theta[j])
    assert np.allclose(np.log10(p), O.log10_pof(theta), rtol=0, atol=1e-13)
    # conjugate-closed sets give equal pof to a root and its conjugate
    assert p[-1] == pytest.approx(p[-2], rel=1e-14)


@pytest.mark.parametrize("log10p,count", [(3.0, 0), (3.999, 0), (4.2, 1), (17.9, 1), (18.3, 2),
                                          (31.5, 2), (32.5, 3), (-2.0, 0)])
def test_extra_root_count_thresholds(log10p, count):
    """A copy for pof > 1e4, a second for pof > 1e18, a third for > 1e32:
    built on the two-root set {1, t} where pof at t is |1 - t|."""
    t = 1.0 + 10.0 ** log10p
    c = O.extra_root_counts(np.array([1.0 + 0j, t]))
    assert c[1] == count
    assert c[0] == 0          # pof(1) = |1 - 1/t| < 1


def test_placement_rule_real_and_pair():
    """First copy at the end; further copies at p + round(k(L-p)/c)."""
    a, b, c, d, e = 10.0, 2e10, 3.0, 4.0, 5.0
    roots = np.array([a, b, c, d, e], dtype=complex)
    counts = O.extra_root_counts(roots)
    # pof(b) = prod |1 - b/x| ~ 1e10^4 / 600 -> log10 ~ 37.2 -> 3 copies
    assert counts[1] == 3 and counts[0] == 0
    out, _ = O.add_stability_roots(roots)
    # p = 1, L = 5: spots 1 + round(4/3) = 2 and 1 + round(8/3) = 4 in the
    # list before insertion, plus the end
    assert list(out.real) == [a, b, b, c, d, b, e, b]
    # a pair is one unit and is never split
    z = 1e12 + 1e11j
    pr = np.array([z, np.conj(z), 2.0, 3.0, 4.0, 5.0], dtype=complex)
    cnt = O.extra_root_counts(pr)
    assert cnt[0] == cnt[1] >= 2
    out2, _ = O.add_stability_roots(pr)
    assert out2.size == pr.size + 2 * cnt[0]
    for i, w in enumerate(out2):
        if w.imag > 0:
            assert out2[i + 1] == np.conj(w)
    assert out2[-2] == z and out2[-1] == np.conj(z)


def test_example7_maxpof_counts_and_accuracy():
    """Example 7: MaxPof (at the largest harmonic Ritz value) and the number
    of extra roots for d = 25 and 40 as printed; the attainable accuracy with
    and without them on either side of the printed values."""
    A = ex7_matrix()
    mv = O.csr_matvec(A)
    rng = np.random.default_rng([7, 1])
    b, v0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    rows = np.loadtxt(os.path.join(GOLD, "example7_stability.txt"))
    polys = {}
    for d, extra, maxpof, ltol, maxerr, side, bound in rows:
        d, extra = int(d), int(extra)
        if d not in polys:
            r, _ = O.gmres_poly(mv, b, d)
            lp = O.log10_pof(r)
            assert abs(lp.max() - np.log10(maxpof)) <= ltol
            assert np.argmax(lp) == np.argmax(np.abs(r))     # at the largest root
            polys[d] = r
        r = polys[d]
        top = r[np.argmax(np.abs(r))]
        stab, counts = O.add_stability_roots(r)
        roots = np.concatenate([r, [top] * extra])        # this row's number of copies
        if extra == counts.sum():
            roots = stab                                   # the procedure's own list
        res, _ = O.pp_eigs(A, b, v0, m=50, k=20, nev=15, roots=roots, rtol=1e-30, max_cycles=25)
        err = min(res.history)
        assert (err >= bound) if side > 0 else (err <= bound), (d, extra, err)
    # the procedure asks for exactly the printed numbers of extra roots
    assert O.extra_root_counts(polys[25]).sum() == 1
    assert O.extra_root_counts(polys[40]).sum() == 2


def test_example7_first_extra_root_at_degree_8():
    """'The test adds a root [for] all d >= 8' (and none below)."""
    A = ex7_matrix()
    mv = O.csr_matvec(A)
    b = np.random.default_rng([7, 1]).standard_normal(A.n)
    for d in (6, 7, 8, 9, 12):
        r, _ = O.gmres_poly(mv, b, d)
        assert (O.extra_root_counts(r).sum() > 0) == (d >= 8), d


def test_example9_double_polynomial_outer_roots():
    """Example 9: with d1 = 5 and pi_1's largest root away from 20000 (here
    19357, the paper's was 19700.5), pi_2(tau(A)) (d2 = 20) has an outstanding
    eigenvalue and Arnoldi(50,20) makes no progress in 50 cycles; the MaxPof
    test on pi_2 asks for extra roots, and with them the 15 wanted pairs
    converge in two cycles."""
    A = ex7_matrix()
    mv = O.csr_matvec(A)
    b = np.random.default_rng(1).standard_normal(A.n)
    v0 = np.random.default_rng([1, 9]).standard_normal(A.n)
    r1, r2 = O.double_poly(mv, b, 5, 20)
    assert 19000 < np.max(np.abs(r1)) < 19900
    assert O.extra_root_counts(r1).sum() == 0
    assert O.extra_root_counts(r2).sum() >= 1
    res, _ = O.pp_eigs(A, b, v0, m=50, k=20, nev=15, roots=(r1, r2), rtol=1e-8, max_cycles=50)
    assert not res.converged and np.sum(res.resid <= 1e-8 * O.infnorm(A)) == 0
    r2s, _ = O.add_stability_roots(r2)
    res2, _ = O.pp_eigs(A, b, v0, m=50, k=20, nev=15, roots=(r1, r2s), rtol=1e-8, max_cycles=50)
    assert res2.converged and res2.cycles <= 2


# ---------------------------------------------------------------- planted mistakes
import oracle.ppa_oracle as P  # noqa: E402


def _pof_swapped(theta):
    theta = np.asarray(theta, dtype=complex)
    return np.array([float(np.prod(np.abs(1.0 - np.delete(theta, j) / theta[j])))
                     for j in range(theta.size)])


def _log10_pof_swapped(theta):
    with np.errstate(divide="ignore"):
        return np.log10(_pof_swapped(theta))


def _counts(fn=np.ceil, base=4.0, step=14.0):
    def extra_root_counts(theta):
        x = (P.log10_pof(theta) - base) / step
        return np.maximum(0, fn(x)).astype(int)
    return extra_root_counts


def _placement(mode):
    def add_stability_roots(theta):
        theta = np.asarray(theta, dtype=complex)
        counts = P.extra_root_counts(theta)
        out = list(theta)
        for j, z in enumerate(theta):
            c = int(counts[j])
            if c == 0 or z.imag < 0.0:
                continue
            unit = [z, np.conj(z)] if z.imag > 0.0 else [z]
            if mode == "front":
                out = unit * c + out
            else:                      # all copies at the end
                out = out + unit * c
        return np.array(out, dtype=complex), counts
    return add_stability_roots


def _fast_counts_pin():
    A = ex7_matrix()
    mv = O.csr_matvec(A)
    b = np.random.default_rng([7, 1]).standard_normal(A.n)
    for d, want in ((25, 1), (40, 2)):
        r, _ = O.gmres_poly(mv, b, d)
        assert O.extra_root_counts(r).sum() == want
        assert abs(O.log10_pof(r).max() - {25: 16.807, 40: 28.309}[d]) <= 0.25


STAB_PINS = [test_pof_is_scaled_derivative,
             *[(lambda a=a, c=c: test_extra_root_count_thresholds(a, c))
               for a, c in [(3.0, 0), (3.999, 0), (4.2, 1), (17.9, 1), (18.3, 2), (32.5, 3)]],
             test_placement_rule_real_and_pair, test_example7_first_extra_root_at_degree_8,
             _fast_counts_pin]

STAB_MUTANTS = {
    "pof: ratio inverted": [("pof", _pof_swapped), ("log10_pof", _log10_pof_swapped)],
    "count: floor instead of ceil": [("extra_root_counts", _counts(fn=np.floor))],
    "count: threshold 1e3": [("extra_root_counts", _counts(base=3.0))],
    "count: one copy per 1e10": [("extra_root_counts", _counts(step=10.0))],
    "placement: copies at the front": [("add_stability_roots", _placement("front"))],
    "placement: all copies at the end": [("add_stability_roots", _placement("end"))],
}


@pytest.mark.parametrize("name", list(STAB_MUTANTS))
def test_stability_mutant_is_caught(name, monkeypatch):
    for attr, fn in STAB_MUTANTS[name]:
        monkeypatch.setattr(P, attr, fn)
        monkeypatch.setattr(O, attr, fn)
    failed = 0
    for pin in STAB_PINS:
        try:
            with np.errstate(all="ignore"):
                pin()
        except Exception:
            failed += 1
    assert failed >= 1, f"no pin caught mutant {name!r}"
