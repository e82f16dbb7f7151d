"""Planted mistakes in the oracle (CPU only): each plausible slip -- a dropped
term, a wrong sign or index, a transposed operand -- must make at least one
pin fail.  This shows the pins constrain every step of the oracle."""
import numpy as np
import pytest

import oracle
import oracle.ppa_oracle as P
from tests import test_oracle_arnoldi as TA
from tests import test_oracle_double as TD
from tests import test_oracle_poly as TP

PINS = [
    TP.test_degree_one_closed_form,
    lambda: TP.test_min_residual_matches_least_squares(4),
    TP.test_harmonic_ritz_generalised_eig_route,
    TP.test_table_3_1_printed_rows,
    TP.test_pair_form_equals_complex_product,
    TP.test_diagonal_exact_mpmath,
    lambda: TP.test_leja_matches_brute_force(3),
    TP.test_leja_log_sum_equals_product_form,
    TA.test_config1_laplacian_closed_form,
    lambda: TA.test_dense_brute_force(1, 6),
    TA.test_arnoldi_relation_and_orthogonality,
    TA.test_restart_keeps_wanted_ritz_values,
    TA.test_restart_with_pair_at_boundary,
    TA.test_example6_one_cycle_counts,
    TD.test_composite_spectral_mapping_diagonal,
    TD.test_second_polynomial_is_min_residual_on_tau,
]


def _harmonic_no_h2(Hbar):
    d = Hbar.shape[1]
    return np.linalg.eigvals(Hbar[:d, :d])


def _harmonic_untransposed(Hbar):
    d = Hbar.shape[1]
    Hd = Hbar[:d, :d]
    e = np.zeros(d); e[-1] = 1
    f = np.linalg.solve(Hd, e)
    return np.linalg.eigvals(Hd + Hbar[d, d - 1] ** 2 * np.outer(f, e))


def _harmonic_f_in_row(Hbar):
    d = Hbar.shape[1]
    Hd = Hbar[:d, :d]
    e = np.zeros(d); e[-1] = 1
    f = np.linalg.solve(Hd.T, e)
    return np.linalg.eigvals(Hd + Hbar[d, d - 1] ** 2 * np.outer(e, f))


def _make_apply(sign=1.0, qmode="mod"):
    def apply_poly(matvec, roots, v, cnt=None, op_mvps=1):
        w = np.array(v, dtype=float)
        i = 0
        while i < len(roots):
            t = roots[i]
            if t.imag == 0:
                w = w - matvec(w) / t.real
                i += 1
            else:
                a = t.real
                q = a * a + t.imag ** 2 if qmode == "mod" else a * a - t.imag ** 2
                s = 2 * a * w - sign * matvec(w)
                w = w - matvec(s) / q
                i += 2
            if cnt is not None:
                cnt.mvps += op_mvps
        return w
    return apply_poly


def _leja_min_first(theta):
    o = P.__dict__["_orig_leja"](theta)
    return o[::-1].copy()


def _sort_by_modulus(nu, target=1.0):
    nu = np.asarray(nu, dtype=complex)
    return np.lexsort((nu.real, -nu.imag, np.abs(nu)))


def _keep_always_k(nu_sorted, k):
    return k


MUTANTS = {
    "harmonic: drop h^2 f e_d^T term": ("harmonic_ritz", _harmonic_no_h2),
    "harmonic: H_d instead of H_d^T": ("harmonic_ritz", _harmonic_untransposed),
    "harmonic: f e_d^T transposed": ("harmonic_ritz", _harmonic_f_in_row),
    "pair: sign of A w flipped": ("apply_poly", _make_apply(sign=-1.0)),
    "pair: |theta|^2 as a^2 - b^2": ("apply_poly", _make_apply(qmode="bad")),
    "leja: reversed order": ("leja_order", _leja_min_first),
    "ritz: sorted by |nu| not |1-nu|": ("sort_ritz", _sort_by_modulus),
}


@pytest.mark.parametrize("name", [
    "harmonic: drop h^2 f e_d^T term", "harmonic: H_d instead of H_d^T",
    "harmonic: f e_d^T transposed", "pair: sign of A w flipped",
    "pair: |theta|^2 as a^2 - b^2", "leja: reversed order",
    "ritz: sorted by |nu| not |1-nu|", "restart: H_m transposed in projection",
    "restart: spike row from the wrong row of Q", "restart: k -> k never reduced for pairs",
    "restart: pair split, real parts kept"])
def test_mutant_is_caught(name, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setitem(P.__dict__, "_orig_leja", P.leja_order)
    monkeypatch.setattr(P, attr, fn)
    if hasattr(oracle, attr):
        monkeypatch.setattr(oracle, attr, fn)
    failed = 0
    for pin in PINS:
        try:
            with np.errstate(all="ignore"):
                pin()
        except Exception:
            failed += 1
    assert failed >= 1, f"no pin caught mutant {name!r}"


def _restart_factory(kind):
    def restart(V, H, G, nu, k, m):
        kk = P.keep_count(nu, k)
        cols = []
        for i in range(kk):
            if nu[i].imag == 0.0:
                cols.append(G[:, i].real)
            elif nu[i].imag > 0.0:
                cols.append(G[:, i].real)
                cols.append(G[:, i].imag)
        if kind == "split_pair":
            kk = k
            cols = [G[:, i].real for i in range(k)]
        Q, _ = np.linalg.qr(np.array(cols).T)
        Vk = V[:, :m] @ Q
        vnext = V[:, m].copy()
        hm = H[m, m - 1]
        Hk = Q.T @ H[:m, :m] @ Q if kind != "transposed" else Q.T @ H[:m, :m].T @ Q
        V[:] = 0.0
        H[:] = 0.0
        V[:, :kk] = Vk
        V[:, kk] = vnext
        H[:kk, :kk] = Hk
        H[kk, :kk] = hm * (Q[0, :] if kind == "spike_row" else Q[m - 1, :])
        return kk
    return restart


MUTANTS["restart: H_m transposed in projection"] = ("thick_restart", _restart_factory("transposed"))
MUTANTS["restart: spike row from the wrong row of Q"] = ("thick_restart", _restart_factory("spike_row"))
MUTANTS["restart: k -> k never reduced for pairs"] = ("keep_count", _keep_always_k)
MUTANTS["restart: pair split, real parts kept"] = ("thick_restart", _restart_factory("split_pair"))
