"""FP64 oracle for polynomial preconditioned Arnoldi (arXiv:1806.08020).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

Every function follows a passage of the paper:

* ``gmres_cycle``      -- section 2, algorithm "Polynomial Preconditioned
                          Arnoldi", step 1(a): one cycle of GMRES(d), i.e. d
                          Arnoldi steps A V_d = V_{d+1} Hbar_{d+1,d}.
* ``harmonic_ritz``    -- same algorithm, step 1(b): eigenvalues of
                          H_d + h_{d+1,d}^2 f e_d^T with f = H_d^{-*} e_d.
* ``leja_order``       -- step 1(c): modified Leja ordering with sums of
                          logarithms in place of products.
* ``apply_poly``       -- eq. (2.1) / step 2: pi(A) v = prod_i (I - A/theta_i) v
                          in Leja order, conjugate pairs applied together in
                          real arithmetic.
* ``thick_restart_arnoldi`` -- step 2 and section 4: Arnoldi(m,k), thick
                          restart with exact shifts, one reorthogonalisation
                          pass, k -> k-1 to keep conjugate pairs whole,
                          convergence tested on A with Rayleigh quotients.
* ``double_poly`` / ``apply_double`` -- section 8: tau = 1 - pi_1, pi_2 from
                          GMRES on tau(A), Arnoldi on pi_2(tau(A)).
* ``Counters``         -- section 4: mvps, dot products, vops and
                          cost = nnzr * mvps + vops.

Readings of points the paper leaves open are listed in the design notes and
repeated at the function that adopts them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

__all__ = [
    "Counters", "csr_matvec", "infnorm", "cgs2", "gmres_cycle", "harmonic_ritz",
    "leja_order", "gmres_poly", "apply_poly", "tau_apply", "double_poly",
    "apply_double", "ArnoldiResult", "thick_restart_arnoldi", "pp_eigs",
    "sort_ritz", "keep_count", "thick_restart", "BREAKDOWN_TOL",
    "pof", "log10_pof", "extra_root_counts", "add_stability_roots",
    "damped_start", "gmres_poly_two", "ideal_order_condition", "order_test_quotients",
    "damping_heuristic", "harmonic_projection", "harmonic_restart", "arnoldi_extend_dcgs2",
]

# Breakdown rule (reading): an Arnoldi/GMRES step breaks down when the norm
# left after orthogonalisation is at most BREAKDOWN_TOL times the norm of the
# vector that entered it.
BREAKDOWN_TOL = 1e-14


@dataclass
class Counters:
    """Operation counts of section 4: matrix-vector products with A, dot
    products, length-n vector operations (dots, axpys, scalings) and
    cost = nnzr * mvps + vops."""
    mvps: int = 0
    dots: int = 0
    vops: int = 0

    def cost(self, nnzr: float) -> float:
        return nnzr * self.mvps + self.vops


# --------------------------------------------------------------------------
# sparse helpers (library primitives)
# --------------------------------------------------------------------------
def csr_matvec(csr):
    """y = A x through SciPy's CSR product (a library primitive)."""
    S = csr.to_scipy()
    return lambda x: S @ x


def infnorm(csr) -> float:
    """||A||_inf, the largest absolute row sum (reading of the norm in
    rtol = ||A|| 1e-8, section 4).  Each stored entry is added to the sum of
    the row it belongs to, so empty rows (first, interior or last) sum to 0."""
    n = int(csr.n)
    if n == 0:
        return 0.0
    rp = np.asarray(csr.rowptr, dtype=np.int64)
    row_of_entry = np.repeat(np.arange(n), np.diff(rp))
    a = np.abs(np.asarray(csr.vals, dtype=np.float64)[: rp[-1]])
    rs = np.bincount(row_of_entry, weights=a, minlength=n)
    return float(rs.max())


# --------------------------------------------------------------------------
# Classical Gram-Schmidt with one reorthogonalisation pass (section 4)
# --------------------------------------------------------------------------
def cgs2(V: np.ndarray, w: np.ndarray, cnt: Counters | None = None):
    """Classical Gram-Schmidt twice against the columns of V.

    Returns (h, w_orth, beta) with h = V^T w accumulated over both passes and
    beta = ||w_orth||."""
    j = V.shape[1]
    h = V.T @ w
    w = w - V @ h
    h2 = V.T @ w
    w = w - V @ h2
    beta = float(np.linalg.norm(w))
    if cnt is not None:
        cnt.dots += 2 * j + 1
        cnt.vops += 4 * j + 2          # 2j dots, 2j axpys, 1 norm, 1 scaling
    return h + h2, w, beta


def arnoldi_extend_dcgs2(op, V: np.ndarray, H: np.ndarray, j0: int, m: int,
                         cnt: Counters | None = None):
    """Arnoldi steps j0..m-1 with Gram-Schmidt and one reorthogonalisation
    pass, the reorthogonalisation delayed by one step so that each step needs
    one block of inner products (a low-synchronisation form of the paper's
    Gram-Schmidt with reorthogonalisation; the paper names communication-
    avoiding variants as future work in section 9).

    V[:, :j0+1] must be orthonormal and H[:j0+1, :j0] hold the projected
    matrix so far.  Step j0 is a plain first pass:
        z = op(q_j0), h = Q^T z, u = z - Q h  (u: once-orthogonalised).
    Step j (j0 < j <= m), with Q = V[:, :j] and u the candidate for q_j:
        a = Q^T u                      (the delayed second pass of z_{j-1})
        beta = sqrt(u^T u - a^T a),    q_j = (u - Q a) / beta
        H[:j, j-1] += a,  H[j, j-1] = beta
    and, while j < m, the next first pass without applying op to q_j:
        w = op(u),  b = Q^T w
        op(q_j) = (w - op(Q) a) / beta = (w - V[:, :j+1] c) / beta,  c = H[:j+1, :j] a
        h = V[:, :j+1]^T op(q_j):  h[:j] = (b - c[:j]) / beta,
                                   h[j]  = ((u^T w - a^T b) / beta - c[j]) / beta
        u_next = op(q_j) - V[:, :j+1] h = w / beta - gamma u - Q g,
            gamma = (c[j] / beta + h[j]) / beta,  g = c[:j] / beta + h[:j] - gamma a.
    Breakdown at step j when beta <= BREAKDOWN_TOL * ||z_{j-1}|| with
    ||z_{j-1}||^2 = ||h_{j-1}||^2 + u^T u (as in ``cgs2`` callers).

    Returns (mc, broke): the basis size reached and whether it broke down."""
    w = op(V[:, j0])
    Q = V[:, : j0 + 1]
    h = Q.T @ w
    H[: j0 + 1, j0] = h
    u = w - Q @ h
    hsq = float(h @ h)
    if cnt is not None:
        cnt.dots += j0 + 1
        cnt.vops += j0 + 1
    for j in range(j0 + 1, m + 1):
        Q = V[:, :j]
        a = Q.T @ u
        uu = float(u @ u)
        beta = float(np.sqrt(max(uu - float(a @ a), 0.0)))
        H[:j, j - 1] += a
        if beta <= BREAKDOWN_TOL * np.sqrt(hsq + uu):
            H[j, j - 1] = 0.0
            return j, True
        H[j, j - 1] = beta
        V[:, j] = (u - Q @ a) / beta
        if cnt is not None:
            cnt.dots += j + 1
            cnt.vops += j + 1
        if j == m:
            break
        w = op(u)
        b = Q.T @ w
        uw = float(u @ w)
        c = H[: j + 1, :j] @ a
        htop = (b - c[:j]) / beta
        hj = ((uw - float(a @ b)) / beta - c[j]) / beta
        H[:j, j] = htop
        H[j, j] = hj
        gamma = (c[j] / beta + hj) / beta
        g = c[:j] / beta + htop - gamma * a
        u = w / beta - gamma * u - Q @ g
        hsq = float(htop @ htop) + hj * hj
        if cnt is not None:
            cnt.dots += j + 1
            cnt.vops += j + 2
    return m, False


# --------------------------------------------------------------------------
# Section 2, step 1: construction of the GMRES polynomial
# --------------------------------------------------------------------------
def gmres_cycle(matvec, b: np.ndarray, d: int, cnt: Counters | None = None):
    """Step 1(a): one cycle of GMRES(d) -- d Arnoldi steps from b giving
    A V_d = V_{d+1} Hbar_{d+1,d}.  Only Hbar is needed for the roots.

    Returns (V, Hbar, d_eff).  If step j breaks down (lucky breakdown: the
    Krylov space is invariant) the effective degree is j and Hbar has a zero
    last row (reading)."""
    n = b.size
    V = np.zeros((n, d + 1))
    H = np.zeros((d + 1, d))
    V[:, 0] = b / np.linalg.norm(b)
    for j in range(d):
        w = matvec(V[:, j])
        if cnt is not None:
            cnt.mvps += 1
        w0 = float(np.linalg.norm(w))
        h, w, beta = cgs2(V[:, : j + 1], w, cnt)
        H[: j + 1, j] = h
        if beta <= BREAKDOWN_TOL * w0:
            Hb = np.zeros((j + 2, j + 1))
            Hb[: j + 1, :] = H[: j + 1, : j + 1]
            return V[:, : j + 2], Hb, j + 1
        H[j + 1, j] = beta
        V[:, j + 1] = w / beta
    return V, H, d


def harmonic_ritz(Hbar: np.ndarray) -> np.ndarray:
    """Step 1(b): harmonic Ritz values, the roots of the GMRES polynomial.

    With Hbar of size (d+1) x d, they are the eigenvalues of
    H_d + h_{d+1,d}^2 f e_d^T where f solves H_d^* f = e_d (H real, so
    H_d^* = H_d^T)."""
    d = Hbar.shape[1]
    Hd = Hbar[:d, :d]
    h = Hbar[d, d - 1]
    e_d = np.zeros(d)
    e_d[-1] = 1.0
    f = np.linalg.solve(Hd.T, e_d)
    M = Hd + (h * h) * np.outer(f, e_d)
    return np.linalg.eigvals(M)


def leja_order(theta: np.ndarray) -> np.ndarray:
    """Step 1(c): modified Leja ordering of a conjugate-closed root set,
    using sums of logarithms of distances in place of products.

    Reading of the details (the cited algorithm is not restated in the
    paper):
      * candidates are pre-sorted by (Re, Im) ascending; a complex pair is
        represented by its member with Im > 0;
      * the first root has the largest modulus (ties: a real root first,
        then the larger real part);
      * each next root maximises sum_{c chosen} log|z - c| over the
        remaining candidates (ties: the earliest in pre-sorted order);
      * when a complex root is chosen its conjugate follows at once;
      * roots whose score is -inf (exact copies of chosen roots) are
        appended last in pre-sorted order.
    """
    theta = np.asarray(theta, dtype=complex)
    pts = theta[np.lexsort((theta.imag, theta.real))]
    reps = [z for z in pts if z.imag >= 0.0]
    n_neg = int(np.sum(pts.imag < 0.0))
    n_pos = int(np.sum(pts.imag > 0.0))
    if n_neg != n_pos:
        raise ValueError("root set is not closed under conjugation")
    out: list[complex] = []

    def take(i):
        z = reps.pop(i)
        out.append(z)
        if z.imag > 0.0:
            out.append(np.conj(z))

    if not reps:
        return np.array([], dtype=complex)
    mods = np.array([abs(z) for z in reps])
    best = None
    for i, z in enumerate(reps):
        if mods[i] != mods.max():
            continue
        key = (0 if z.imag == 0.0 else 1, -z.real)
        if best is None or key < best[0]:
            best = (key, i)
    take(best[1])
    while reps:
        with np.errstate(divide="ignore"):
            scores = np.array([np.sum(np.log(np.abs(z - np.array(out)))) for z in reps])
        i = int(np.argmax(scores))
        if scores[i] == -np.inf:
            while reps:
                take(0)
            break
        take(i)
    return np.array(out, dtype=complex)


def gmres_poly(matvec, b: np.ndarray, d: int, cnt: Counters | None = None):
    """Step 1 of the algorithm: GMRES(d) -> harmonic Ritz values -> Leja.
    Returns (roots in Leja order, effective degree)."""
    _, Hbar, d_eff = gmres_cycle(matvec, b, d, cnt)
    return leja_order(harmonic_ritz(Hbar)), d_eff


# --------------------------------------------------------------------------
# eq. (2.1): pi(A) v in factored form
# --------------------------------------------------------------------------
# ---------------------------------------------------------------- start vectors (sections 5, 6)
def damped_start(matvec, b: np.ndarray, power: int = 1, alpha: float = 0.0) -> np.ndarray:
    """Section 6, damped polynomials: the GMRES start vector A^power b, plus
    alpha * b when alpha != 0 (the A b + alpha b family).  Premultiplying by
    A damps b's components along eigenvectors of small eigenvalues, so the
    GMRES polynomial tries less hard to be small there."""
    x = np.array(b, dtype=float)
    for _ in range(power):
        x = matvec(x)
    return x + alpha * np.asarray(b, dtype=float) if alpha != 0.0 else x


def gmres_poly_two(matvec, b1: np.ndarray, b2: np.ndarray, d: int, cnt: Counters | None = None):
    """Section 5, 'Polynomial determined by two starting vectors': b1, b2
    scaled to norm 1/sqrt(2) each, one GMRES(d) cycle on the block-diagonal
    system diag(A, A) of dimension 2n from [b1; b2]; its polynomial is
    applied to A.  Returns (roots in Leja order, effective degree)."""
    n = b1.size
    bh = np.concatenate([b1 / (np.sqrt(2.0) * np.linalg.norm(b1)),
                         b2 / (np.sqrt(2.0) * np.linalg.norm(b2))])

    def mv2(x):
        return np.concatenate([matvec(x[:n]), matvec(x[n:])])
    return gmres_poly(mv2, bh, d, cnt)


def ideal_order_condition(mu: np.ndarray, nev: int, k: int) -> bool:
    """Section 6, step 4: |mu_1| <= ... <= |mu_nev| < min_{nev < j <= k} |mu_j|,
    for Rayleigh quotients listed in the order of |1 - nu_j|."""
    a = np.abs(np.asarray(mu)[:k])
    mono = all(a[i] <= a[i + 1] for i in range(nev - 1))
    return bool(mono and (nev == k or a[nev - 1] < a[nev:k].min()))


def order_test_quotients(csr, roots, b: np.ndarray, m: int, k: int) -> np.ndarray:
    """Section 6, steps 1-3: one Arnoldi(m,k) cycle on pi(A) from b, Ritz
    values nu_j ordered by |1 - nu_j|, and mu_j = y_j^* A y_j for the first k
    (unit Ritz vectors), returned in that order."""
    amv = csr_matvec(csr)
    op = (lambda x: apply_poly(amv, roots, x))
    res = thick_restart_arnoldi(op, amv, b, m, k, k, 0.0, 1)
    o = sort_ritz(res.nu)
    return res.mu[o]


def damping_heuristic(csr, b: np.ndarray, d: int, m: int, k: int, nev: int):
    """Section 6, 'Heuristic for damping b and adjusting d'.  Build pi from b
    and test the Ideal Order Condition on one Arnoldi(m,k) cycle; if it
    fails, rebuild pi from A b and test again; while it still fails, halve d
    (keeping the damped start vector) and test again, down to d = 1.
    Returns (roots, info) with info = dict(d, damped, attempts, held)."""
    amv = csr_matvec(csr)
    start, damped, attempts = np.array(b, dtype=float), False, 0
    while True:
        roots, _ = gmres_poly(amv, start, d)
        attempts += 1
        held = ideal_order_condition(order_test_quotients(csr, roots, b, m, k), nev, k)
        if held or d == 1:
            return roots, dict(d=d, damped=damped, attempts=attempts, held=held)
        if not damped:
            start, damped = damped_start(amv, b, 1), True
        else:
            d = d // 2


# ---------------------------------------------------------------- stability (section 7)
def pof(theta: np.ndarray) -> np.ndarray:
    """Section 7: pof(j) = prod_{i != j} |1 - theta_j / theta_i|, the product
    of the other factors of pi evaluated at theta_j (so |pi'(theta_j)| =
    pof(j) / |theta_j|).  Written as the definition: a product, which may
    overflow to inf for high degrees (log10_pof is the same quantity as a sum
    of logarithms)."""
    theta = np.asarray(theta, dtype=complex)
    out = np.empty(theta.size)
    for j in range(theta.size):
        others = np.delete(theta, j)
        out[j] = float(np.prod(np.abs(1.0 - theta[j] / others)))
    return out


def log10_pof(theta: np.ndarray) -> np.ndarray:
    """log10 pof(j) = sum_{i != j} log10 |1 - theta_j / theta_i| (no overflow;
    -inf when theta_j repeats)."""
    theta = np.asarray(theta, dtype=complex)
    out = np.empty(theta.size)
    with np.errstate(divide="ignore"):
        for j in range(theta.size):
            others = np.delete(theta, j)
            out[j] = float(np.sum(np.log10(np.abs(1.0 - theta[j] / others))))
    return out


def extra_root_counts(theta: np.ndarray) -> np.ndarray:
    """Section 7, 'Adding roots for stability', step 2-3 count: one more copy
    of theta_j for every factor 1e14 by which pof(j) exceeds 1e4, i.e.
    ceil((log10 pof(j) - 4) / 14), never negative (reading: a copy is added
    only when pof(j) exceeds 1e4, a second when it exceeds 1e18, ...)."""
    x = (log10_pof(theta) - 4.0) / 14.0
    return np.maximum(0, np.ceil(x)).astype(int)


def add_stability_roots(theta: np.ndarray):
    """Section 7, 'Adding roots for stability', on a root list in modified
    Leja order.  For each root in list order (a conjugate pair as one unit,
    at its Im > 0 member) with c = extra_root_counts > 0: the first copy goes
    to the end of the current list; the other c - 1 are inserted at the
    positions p + round(k (L - p) / c), k = 1..c-1, spaced evenly between the
    root's position p and the end of the current list (length L before
    this root's copies), never between the two members of a pair.  pof is
    evaluated once, on the original list.  Returns (new list, counts)."""
    theta = np.asarray(theta, dtype=complex)
    counts = extra_root_counts(theta)
    out = list(theta)
    for j, z in enumerate(theta):
        c = int(counts[j])
        if c == 0 or z.imag < 0.0:
            continue
        unit = [z, np.conj(z)] if z.imag > 0.0 else [z]
        p = next(i for i, w in enumerate(out) if w == z)
        L = len(out)
        spots = []
        for kk in range(1, c):
            q = p + int(np.floor(kk * (L - p) / c + 0.5))
            if 0 < q < len(out) and out[q - 1].imag > 0.0 and out[q] == np.conj(out[q - 1]):
                q += 1   # not between a pair's members
            spots.append(q)
        out = out + unit
        for q in sorted(spots, reverse=True):
            out[q:q] = unit
    return np.array(out, dtype=complex), counts


def apply_poly(matvec, roots: np.ndarray, v: np.ndarray, cnt: Counters | None = None,
               op_mvps: int = 1):
    """pi(A) v = prod_i (I - A/theta_i) v, factors in the given (Leja) order.

    A real root theta gives w <- w - (1/theta) A w.  A conjugate pair
    theta = a +/- ib (kept together, section 7) is applied in real
    arithmetic through (I - A/theta)(I - A/conj(theta))
    = I - (2a/|theta|^2) A + (1/|theta|^2) A^2, evaluated as
    s = 2a w - A w,  w <- w - (1/|theta|^2) A s.

    ``op_mvps`` is the number of products with A that one call of
    ``matvec`` costs (0 when ``matvec`` counts its own, as tau(A) does)."""
    w = np.array(v, dtype=np.float64, copy=True)
    i = 0
    roots = np.asarray(roots, dtype=complex)
    while i < roots.size:
        t = roots[i]
        if t.imag == 0.0:
            w = w - matvec(w) / t.real
            if cnt is not None:
                cnt.mvps += op_mvps
                cnt.vops += 1
            i += 1
        else:
            if i + 1 >= roots.size or roots[i + 1] != np.conj(t):
                raise ValueError("complex root without its conjugate next to it")
            a = t.real
            q = t.real * t.real + t.imag * t.imag
            s = 2.0 * a * w - matvec(w)
            w = w - matvec(s) / q
            if cnt is not None:
                cnt.mvps += 2 * op_mvps
                cnt.vops += 2
            i += 2
    return w


# --------------------------------------------------------------------------
# Section 8: double polynomial preconditioning
# --------------------------------------------------------------------------
def tau_apply(matvec, roots1, x, cnt: Counters | None = None):
    """tau(A) x with tau = 1 - pi_1:  x - pi_1(A) x."""
    if cnt is not None:
        cnt.vops += 1
    return x - apply_poly(matvec, roots1, x, cnt)


def double_poly(matvec, b: np.ndarray, d1: int, d2: int, cnt: Counters | None = None):
    """pi_1 of degree d1 from GMRES on A, then pi_2 of degree d2 from GMRES on
    tau(A) = I - pi_1(A), both from the same start vector b (reading).
    Returns (roots1, roots2)."""
    r1, _ = gmres_poly(matvec, b, d1, cnt)
    c2 = Counters()
    r2, _ = gmres_poly(lambda x: tau_apply(matvec, r1, x, cnt), b, d2, c2)
    if cnt is not None:          # tau(A) counts its own products with A
        cnt.dots += c2.dots
        cnt.vops += c2.vops
    return r1, r2


def apply_double(matvec, roots1, roots2, v, cnt: Counters | None = None):
    """pi_2(tau(A)) v, composite degree d1*d2."""
    return apply_poly(lambda x: tau_apply(matvec, roots1, x, cnt), roots2, v, cnt, op_mvps=0)


# --------------------------------------------------------------------------
# Section 2 step 2 and section 4: thick-restarted Arnoldi(m,k) on pi(A)
# --------------------------------------------------------------------------
def sort_ritz(nu: np.ndarray, target: float = 1.0) -> np.ndarray:
    """Order Ritz values of pi(A) by increasing |1 - nu| (section 4).
    Ties: larger imaginary part first (so a conjugate pair is adjacent with
    Im > 0 first), then smaller real part.  ``target = 0`` orders by |nu|,
    which is standard Arnoldi on A seeking the smallest magnitudes (the
    paper's d = 0 rows)."""
    nu = np.asarray(nu, dtype=complex)
    return np.lexsort((nu.real, -nu.imag, np.abs(target - nu)))


def keep_count(nu_sorted: np.ndarray, k: int) -> int:
    """Number of Ritz vectors kept at a restart: k, or k-1 when the k-th and
    (k+1)-th sorted values are a conjugate pair (section 4 footnote)."""
    if k < len(nu_sorted) and nu_sorted[k - 1].imag > 0.0:
        return k - 1
    return k


def thick_restart(V: np.ndarray, H: np.ndarray, G: np.ndarray, nu: np.ndarray, k: int, m: int) -> int:
    """Thick restart with exact shifts (section 2 step 2, section 4), in place.

    Keeps the first k sorted Ritz vectors (k-1 if that would split a
    conjugate pair) as a real orthonormal basis Q of [Re g, Im g] columns,
    then V_k <- V_m Q, v_{k+1} <- v_{m+1}, H_k <- Q^T H_m Q and the new row
    k+1 holds h_{m+1,m} e_m^T Q.  Returns the number of kept vectors."""
    kk = keep_count(nu, k)
    cols = []
    for i in range(kk):
        if nu[i].imag == 0.0:
            cols.append(G[:, i].real)
        elif nu[i].imag > 0.0:
            cols.append(G[:, i].real)
            cols.append(G[:, i].imag)
    Q, _ = np.linalg.qr(np.array(cols).T)
    Vk = V[:, :m] @ Q
    vnext = V[:, m].copy()
    hm = H[m, m - 1]
    Hk = Q.T @ H[:m, :m] @ Q
    V[:] = 0.0
    H[:] = 0.0
    V[:, :kk] = Vk
    V[:, kk] = vnext
    H[:kk, :kk] = Hk
    H[kk, :kk] = hm * Q[m - 1, :]
    return kk


def harmonic_projection(Hm: np.ndarray, hm: float, target: float):
    """Harmonic Ritz pairs of the projected operator with respect to the
    target tau (the harmonic Arnoldi method the paper uses in section 4,
    Example 2): f = (H_m - tau I)^{-T} e_m and the eigenpairs (theta, g) of
    H_m + h_{m+1,m}^2 f e_m^T.  Returns (theta, G, f)."""
    m = Hm.shape[0]
    e = np.zeros(m)
    e[-1] = 1.0
    f = np.linalg.solve((Hm - target * np.eye(m)).T, e)
    theta, G = np.linalg.eig(Hm + hm * hm * np.outer(f, e))
    return theta, G, f


def harmonic_restart(V: np.ndarray, H: np.ndarray, G: np.ndarray, theta: np.ndarray,
                     f: np.ndarray, k: int, m: int) -> int:
    """Thick restart keeping harmonic Ritz vectors, in place.  Every harmonic
    Ritz pair (theta, y = V_m g) has residual op(y) - theta y parallel to
    w = v_{m+1} - h_{m+1,m} V_m f, so span{y_1..y_kk, w} carries a
    Krylov-like relation: with Q a real orthonormal basis of the kept g's
    (k-1 when a pair would be split) and w_hat = [-h f; 1] orthonormalised
    against [Q; 0], the new basis is V_{m+1} [[Q, *], [0, *]] (w_hat last)
    and the new projected block is [Q; 0 | w_hat]^T H_bar_m Q, a full
    (kk+1) x kk matrix.  Returns the number of kept vectors."""
    kk = keep_count(theta, k)
    cols = []
    for i in range(kk):
        if theta[i].imag == 0.0:
            cols.append(G[:, i].real)
        elif theta[i].imag > 0.0:
            cols.append(G[:, i].real)
            cols.append(G[:, i].imag)
    Q, _ = np.linalg.qr(np.array(cols).T)
    hm = H[m, m - 1]
    Qh = np.vstack([Q, np.zeros((1, kk))])
    w = np.concatenate([-hm * f.real, [1.0]])
    for _ in range(2):
        w = w - Qh @ (Qh.T @ w)
    w = w / np.linalg.norm(w)
    Qp = np.hstack([Qh, w[:, None]])
    Hn = Qp.T @ H[: m + 1, :m] @ Q
    Vn = V[:, : m + 1] @ Qp
    V[:] = 0.0
    H[:] = 0.0
    V[:, : kk + 1] = Vn
    H[: kk + 1, :kk] = Hn
    return kk


@dataclass
class ArnoldiResult:
    mu: np.ndarray            # eigenvalue estimates of A (Rayleigh quotients), sorted by |mu|
    resid: np.ndarray         # ||A y - mu y|| for each returned pair
    Y: np.ndarray             # unit Ritz vectors (complex), columns match mu
    converged: bool
    cycles: int
    counters: Counters = field(default_factory=Counters)
    nu: np.ndarray | None = None      # Ritz values of pi(A) of the wanted pairs
    history: list = field(default_factory=list)   # max wanted residual per cycle
    breakdown: bool = False


def _ritz_test(Vm, g_cols, amatvec, cnt):
    """Unit Ritz vectors y = V_m g / ||V_m g||, Rayleigh quotients
    mu = y^* A y and residual norms ||A y - mu y|| (section 4)."""
    mus, res, Ys = [], [], []
    for g in g_cols:
        y = Vm @ g
        y = y / np.linalg.norm(y)
        if np.iscomplexobj(y) and np.any(y.imag != 0.0):
            Ay = amatvec(y.real) + 1j * amatvec(y.imag)
            if cnt is not None:
                cnt.mvps += 2
        else:
            y = y.real.astype(complex)
            Ay = amatvec(y.real).astype(complex)
            if cnt is not None:
                cnt.mvps += 1
        mu = np.vdot(y, Ay)
        r = np.linalg.norm(Ay - mu * y)
        mus.append(mu); res.append(r); Ys.append(y)
    return np.array(mus), np.array(res), np.array(Ys).T


def thick_restart_arnoldi(op, amatvec, v0: np.ndarray, m: int, k: int, nev: int,
                          rtol_abs: float, max_cycles: int,
                          cnt: Counters | None = None, hook=None,
                          target: float = 1.0, shift: float = 0.0,
                          harmonic: bool = False, ortho: str = "cgs2") -> ArnoldiResult:
    """Thick-restarted Arnoldi(m,k) with exact shifts on the operator ``op``
    (pi(A) or pi_2(tau(A))), convergence tested on A (section 4).

    Cycle: extend the basis to m vectors with Gram-Schmidt plus one
    reorthogonalisation pass; take eigenpairs (nu, g) of H_m; order by
    |1 - nu|; test the first nev with y = V_m g/||V_m g||, mu = y^* A y,
    ||A y - mu y|| <= rtol_abs; if not converged keep the first k (k-1 if a
    conjugate pair would be split) as a real orthonormal basis Q of their
    Ritz vectors, V_k <- V_m Q, v_{k+1} <- v_{m+1},
    H_k <- Q^T H_m Q with row k+1 equal to h_{m+1,m} e_m^T Q, and continue.
    ``harmonic``: the pairs are harmonic Ritz pairs with respect to the
    target (harmonic_projection) and the restart keeps harmonic Ritz vectors
    (harmonic_restart); the test is unchanged.
    ``ortho``: "cgs2" (Gram-Schmidt with one reorthogonalisation pass, as in
    the paper) or "dcgs2" (the same with the reorthogonalisation delayed by
    one step, ``arnoldi_extend_dcgs2``).

    ``hook(event, V, H, j)``, if given, sees copies of the basis and the
    projected matrix at the end of each cycle (event "cycle", j = basis
    size) and after each restart (event "restart", j = vectors kept); it is
    an inspection point for tests and changes nothing.
    """
    cnt = cnt if cnt is not None else Counters()
    n = v0.size
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m))
    V[:, 0] = v0 / np.linalg.norm(v0)
    j0 = 0
    history = []
    res = None
    for cycle in range(1, max_cycles + 1):
        mcyc = m
        broke = False
        if ortho == "dcgs2":
            mcyc, broke = arnoldi_extend_dcgs2(op, V, H, j0, m, cnt)
        for j in range(j0, m if ortho != "dcgs2" else j0):
            w = op(V[:, j])
            w0 = float(np.linalg.norm(w))
            h, w, beta = cgs2(V[:, : j + 1], w, cnt)
            H[: j + 1, j] = h
            if beta <= BREAKDOWN_TOL * w0:
                H[j + 1, j] = 0.0
                mcyc = j + 1
                broke = True
                break
            H[j + 1, j] = beta
            V[:, j + 1] = w / beta
        if hook is not None:
            hook("cycle", V.copy(), H.copy(), mcyc)
        Hm = H[:mcyc, :mcyc]
        if harmonic:
            nu, G, fh = harmonic_projection(Hm, H[mcyc, mcyc - 1], target)
        else:
            nu, G = np.linalg.eig(Hm)
        order = sort_ritz(nu, target)
        nu, G = nu[order], G[:, order]
        nw = min(nev, mcyc)
        mu, rr, Y = _ritz_test(V[:, :mcyc], [G[:, i] for i in range(nw)], amatvec, cnt)
        history.append(float(rr.max()) if rr.size else 0.0)
        done = bool(np.all(rr <= rtol_abs)) and nw == nev
        res = (mu, rr, Y, nu[:nw])
        if done or broke or cycle == max_cycles:
            conv = done
            break
        kk = harmonic_restart(V, H, G, nu, fh, k, m) if harmonic else thick_restart(V, H, G, nu, k, m)
        j0 = kk
        if hook is not None:
            hook("restart", V.copy(), H.copy(), kk)
    mu, rr, Y, nus = res
    # returned by distance to the target point of A (the shift; R9)
    o = np.lexsort((mu.imag, mu.real, np.abs(mu - shift)))
    return ArnoldiResult(mu=mu[o], resid=rr[o], Y=Y[:, o], converged=conv, cycles=cycle,
                         counters=cnt, nu=nus[o], history=history, breakdown=broke)


def pp_eigs(csr, b: np.ndarray, v0: np.ndarray, m: int, k: int, nev: int,
            d: int | None = None, d1: int | None = None, d2: int | None = None,
            rtol: float = 1e-8, max_cycles: int = 100, roots=None, hook=None,
            shift: float = 0.0, harmonic: bool = False, ortho: str = "cgs2"):
    """Polynomial preconditioned Arnoldi end to end (section 2 listing;
    section 8 for ``d1, d2``).  rtol is relative: the absolute bound is
    rtol * ||A||_inf.  ``d=0`` runs standard Arnoldi on A.  ``roots`` may
    give a ready root list (single polynomial) or a pair (roots1, roots2).
    ``shift`` = mu (section 2 footnote: for eigenvalues near mu use A - mu I):
    the polynomial is built for and applied to A - mu I, the Rayleigh
    quotients and residuals are those of A (the residual is the same for
    both), and the eigenvalues are returned by their distance to mu.
    ``harmonic`` restarts with harmonic Ritz vectors and ``ortho`` selects the
    Gram-Schmidt form (thick_restart_arnoldi).

    Returns (ArnoldiResult, roots) where roots is a list or a (r1, r2) pair."""
    amv0 = csr_matvec(csr)
    cnt = Counters()
    amv = (lambda x: amv0(x) - shift * x) if shift != 0.0 else amv0

    if roots is not None:
        rts = roots
    elif d1 is not None:
        rts = double_poly(amv, b, d1, d2, cnt)
    elif d:
        rts, _ = gmres_poly(amv, b, d, cnt)
    else:
        rts = None
    if rts is None:
        def op(x):
            cnt.mvps += 1
            return amv(x)
    elif isinstance(rts, tuple):
        r1, r2 = rts
        def op(x):
            return apply_double(amv, r1, r2, x, cnt)
    else:
        def op(x):
            return apply_poly(amv, rts, x, cnt)
    res = thick_restart_arnoldi(op, amv0, v0, m, k, nev, rtol * infnorm(csr), max_cycles, cnt, hook,
                                target=0.0 if rts is None else 1.0, shift=shift, harmonic=harmonic,
                                ortho=ortho)
    return res, rts
