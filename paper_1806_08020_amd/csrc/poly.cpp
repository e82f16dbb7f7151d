// The GMRES polynomial: construction (section 2, step 1) and application in
// factored form (eq. (2.1)), single and double (section 8).
#include <algorithm>
#include <cmath>
#include <limits>

#include "ppa_internal.hpp"

namespace ppa {

// ---------------------------------------------------------------- roots
// Step 1(b): harmonic Ritz values = eig(H_d + h_{d+1,d}^2 f e_d^T) with
// H_d^T f = e_d.  The modified matrix stays upper Hessenberg (only its last
// column changes), so Francis QR applies directly.
std::vector<cplx> harmonic_ritz(int d, const std::vector<double>& Hbar) {
    const int ld = d + 1;
    std::vector<double> Hd((size_t)d * d), HdT((size_t)d * d);
    for (int j = 0; j < d; ++j)
        for (int i = 0; i < d; ++i) {
            Hd[i + (size_t)j * d] = Hbar[i + (size_t)j * ld];
            HdT[j + (size_t)i * d] = Hbar[i + (size_t)j * ld];
        }
    const double h = Hbar[d + (size_t)(d - 1) * ld];
    std::vector<double> f(d, 0.0);
    f[d - 1] = 1.0;
    if (h != 0.0) {
        if (!lu_solve(d, HdT, f)) fail(PPA_ERR_SINGULAR, "harmonic Ritz: H_d is singular (d=%d)", d);
        for (int i = 0; i < d; ++i) Hd[i + (size_t)(d - 1) * d] += h * h * f[i];
    }
    std::vector<cplx> w;
    hessenberg_eigvals(d, Hd, w);
    return w;
}

// Step 1(c): modified Leja ordering with sums of logarithms.  Reading of the
// details: candidates pre-sorted by (Re, Im); a conjugate pair is represented
// by its Im > 0 member and its conjugate follows it at once; the first root
// has the largest modulus (ties: real first, then larger real part); each
// next root maximises sum log|z - c| over the roots already placed (ties: the
// earliest in pre-sorted order); roots scoring -inf (copies of placed roots)
// are appended last in pre-sorted order.
std::vector<cplx> leja_order(const std::vector<cplx>& theta) {
    std::vector<cplx> pts = theta;
    std::stable_sort(pts.begin(), pts.end(), [](const cplx& a, const cplx& b) {
        if (a.real() != b.real()) return a.real() < b.real();
        return a.imag() < b.imag();
    });
    std::vector<cplx> reps;
    int npos = 0, nneg = 0;
    for (const cplx& z : pts) {
        if (z.imag() >= 0.0) reps.push_back(z);
        if (z.imag() > 0.0) ++npos;
        if (z.imag() < 0.0) ++nneg;
    }
    PPA_REQUIRE(npos == nneg, "root set is not closed under conjugation");
    std::vector<cplx> out;
    out.reserve(theta.size());
    auto take = [&](size_t i) {
        const cplx z = reps[i];
        reps.erase(reps.begin() + i);
        out.push_back(z);
        if (z.imag() > 0.0) out.push_back(std::conj(z));
    };
    if (reps.empty()) return out;
    {
        double mx = -1.0;
        for (const cplx& z : reps) mx = std::max(mx, std::abs(z));
        size_t best = reps.size();
        for (size_t i = 0; i < reps.size(); ++i) {
            if (std::abs(reps[i]) != mx) continue;
            if (best == reps.size()) { best = i; continue; }
            const cplx& b = reps[best];
            const int kb = b.imag() == 0.0 ? 0 : 1, ki = reps[i].imag() == 0.0 ? 0 : 1;
            if (ki < kb || (ki == kb && reps[i].real() > b.real())) best = i;
        }
        take(best);
    }
    while (!reps.empty()) {
        size_t best = 0;
        double bs = -std::numeric_limits<double>::infinity();
        bool any = false;
        for (size_t i = 0; i < reps.size(); ++i) {
            double sc = 0.0;
            for (const cplx& c : out) sc += std::log(std::abs(reps[i] - c));
            if (!any || sc > bs) {
                bs = sc;
                best = i;
                any = true;
            }
        }
        if (bs == -std::numeric_limits<double>::infinity()) {
            while (!reps.empty()) take(0);
            break;
        }
        take(best);
    }
    return out;
}

// ---------------------------------------------------------------- apply
// A shifted double polynomial may need one more buffer (the two-step last
// pass below).
int apply_buffers(const Poly& p) { return p.is_double() ? (p.shift != 0.0 ? 7 : 6) : 4; }

void carve_apply(Carver& c, int64_t n, const Poly& p, VecT t, ApplyWs& ws) {
    const size_t es = t == VecT::F64 ? sizeof(double) : sizeof(float);
    for (int i = 0; i < apply_buffers(p); ++i) ws.buf[i] = c.take<char>((size_t)n * es);
}

namespace {

struct Chain {
    const Matrix& A;
    VecT ct;            // chain element type
    hipStream_t s;
    std::vector<void*> pool;
    size_t bytes = 0;
    bool dry = false;   // count bytes only
    double sigma = 0.0; // the operator is A - sigma I
    void pass(double alpha, const void* x, double beta, const void* u, double gamma, const void* z,
              double delta, const void* z2, void* out, VecT out_t) {
        if (dry)
            bytes += fused_spmv_bytes(A, ct, out_t, x, u, z, z2);
        else
            bytes += launch_fused_spmv(A, ct, out_t, alpha, x, beta, u, gamma, z, delta, z2, out, s);
    }
    // two consecutive factor passes as one launch (launch_two_step):
    // s = a1 u + b1 A u, out = a2 x2 + b2 A s (+ g2 s with zs), x2 = s or u
    void pass_two(double a1, double b1, double a2, double b2, double g2, bool zs, bool x2s,
                  const void* u, void* out) {
        if (dry) {
            static char tag_s;
            const void* sp = &tag_s;
            bytes += fused_spmv_bytes(A, ct, ct, u, u, nullptr, nullptr) +
                     fused_spmv_bytes(A, ct, ct, x2s ? sp : u, sp, zs ? sp : nullptr, nullptr);
        } else {
            bytes += launch_two_step(A, ct, a1, b1, a2, b2, g2, zs, x2s, u, out, s);
        }
    }
    void axpy3(double a, const void* x, double b, const void* y, double c, const void* z, void* out,
               VecT out_t) {
        const size_t sin = ct == VecT::F64 ? 8 : 4, sout = out_t == VecT::F64 ? 8 : 4;
        bytes += (size_t)A.n * (sin * (1 + (y != nullptr) + (z != nullptr)) + sout);
        if (!dry) launch_axpy3(A.n, ct, out_t, a, x, b, y, c, z, out, s);
    }
};

// out = c * pi(A) u0 + gamma z + delta z2, factors in order.  `busy` lists
// buffers the caller still needs.
void pi_chain(Chain& ch, const std::vector<cplx>& roots, const void* u0, double c, double gamma,
              const void* z, double delta, const void* z2, void* out, VecT out_t,
              std::initializer_list<const void*> busy_outer) {
    const void* cur = u0;
    const size_t nr = roots.size();
    std::vector<const void*> busy(busy_outer);
    auto pick = [&](const void* a, const void* b) {
        for (void* buf : ch.pool) {
            bool used = buf == a || buf == b || buf == out;
            for (const void* q : busy) used |= (q == buf);
            if (!used) return buf;
        }
        fail(PPA_ERR_INVALID, "internal: apply buffer pool exhausted");
    };
    // With a shift sigma the factors act on A - sigma I; sigma folds into the
    // coefficients of the vector that is also the gathered one:
    //   real:  w - (A - sigma) w / theta = (1 + sigma/theta) w - A w / theta
    //   pair:  s = (2a + sigma) w - A w,  w - (A - sigma) s / q = w - A s / q + (sigma/q) s
    const double sg = ch.sigma;
    // two factors per launch where the matrix has the records for it: two
    // real roots in a row or a conjugate pair, neither the chain's last
    // factor (that one carries the scaling and the epilogue terms)
    const bool two = two_step_on(ch.A, ch.ct);
    size_t i = 0;
    while (i < nr) {
        const cplx t = roots[i];
        const bool pair = t.imag() != 0.0;
        const bool last = (i + (pair ? 2 : 1)) >= nr;
        if (two && !pair && i + 2 < nr && roots[i + 1].imag() == 0.0) {
            const double ib = -1.0 / t.real(), ib2 = -1.0 / roots[i + 1].real();
            void* nx = pick(cur, nullptr);
            ch.pass_two(1.0 - sg * ib, ib, 1.0 - sg * ib2, ib2, 0.0, false, true, cur, nx);
            cur = nx;
            i += 2;
            continue;
        }
        if (two && pair && !last) {
            const double q = t.real() * t.real() + t.imag() * t.imag();
            const double ss = sg / q;
            void* nx = pick(cur, nullptr);
            ch.pass_two(2.0 * t.real() + sg, -1.0, 1.0, -1.0 / q, ss, ss != 0.0, false, cur, nx);
            cur = nx;
            i += 2;
            continue;
        }
        if (!pair) {
            const double ib = -1.0 / t.real();
            const double sx = 1.0 - sg * ib;
            if (last) {
                ch.pass(c * sx, cur, c * ib, cur, gamma, z, delta, z2, out, out_t);
            } else {
                void* nx = pick(cur, nullptr);
                ch.pass(sx, cur, ib, cur, 0.0, nullptr, 0.0, nullptr, nx, ch.ct);
                cur = nx;
            }
            i += 1;
        } else {
            const double a = t.real();
            const double q = t.real() * t.real() + t.imag() * t.imag();
            const double ss = sg / q;
            void* sb = pick(cur, nullptr);
            ch.pass(2.0 * a + sg, cur, -1.0, cur, 0.0, nullptr, 0.0, nullptr, sb, ch.ct);
            if (!last) {
                void* nx = pick(cur, sb);
                ch.pass(1.0, cur, -1.0 / q, sb, ss, ss != 0.0 ? sb : nullptr, 0.0, nullptr, nx, ch.ct);
                cur = nx;
            } else if (ss == 0.0) {
                ch.pass(c, cur, -c / q, sb, gamma, z, delta, z2, out, out_t);
            } else {
                // c w - (c/q) A s + (c sigma/q) s + gamma z + delta z2: merge terms on
                // the same vector, then put the s term in a free slot
                double al = c, g1 = gamma, g2 = delta;
                const void* z1p = z;
                const void* z2p = z2;
                if (z1p == cur) { al += g1; z1p = nullptr; g1 = 0.0; }
                if (z2p == cur) { al += g2; z2p = nullptr; g2 = 0.0; }
                const double es = c * ss;
                if (z1p == sb) {
                    g1 += es;
                } else if (z2p == sb) {
                    g2 += es;
                } else if (z1p == nullptr) {
                    z1p = sb;
                    g1 = es;
                } else if (z2p == nullptr) {
                    z2p = sb;
                    g2 = es;
                } else {
                    // five distinct vectors: the factor first, then the epilogue
                    void* tmp = pick(cur, sb);
                    ch.pass(1.0, cur, -1.0 / q, sb, ss, sb, 0.0, nullptr, tmp, ch.ct);
                    ch.axpy3(al, tmp, g1, z1p, g2, z2p, out, out_t);
                    i += 2;
                    continue;
                }
                ch.pass(al, cur, -c / q, sb, g1, z1p, g2, z2p, out, out_t);
            }
            i += 2;
        }
    }
}

}  // namespace

size_t apply_single_epilogue(const Matrix& A, const std::vector<cplx>& roots, const double* v,
                             double* y, double c, double gamma, const double* z, ApplyWs& ws,
                             hipStream_t s, double sigma) {
    PPA_REQUIRE(!roots.empty(), "apply: empty polynomial");
    Chain ch{A, VecT::F64, s, {}};
    ch.sigma = sigma;
    for (int i = 0; i < 4; ++i) ch.pool.push_back(ws.buf[i]);
    pi_chain(ch, roots, v, c, gamma, z, 0.0, nullptr, y, VecT::F64, {v, z});
    return ch.bytes;
}

namespace {

// pi(A) v0 -> y through the chain's buffer pool (single or double polynomial)
void run_apply(Chain& ch, const Poly& p, const void* v0, VecT vout, void* y) {
    const VecT chain = ch.ct;
    if (!p.is_double()) {
        pi_chain(ch, p.roots, v0, 1.0, 0.0, nullptr, 0.0, nullptr, y, vout, {v0});
        return;
    }
    // pi_2(tau(A)) v with tau = 1 - pi_1 (section 8):
    //  real eta:  w <- (1 - 1/eta) w + (1/eta) pi_1(A) w
    //  pair eta:  s = (2a - 1) w + pi_1(A) w,
    //             w <- w - s/|eta|^2 + (1/|eta|^2) pi_1(A) s
    const void* w = v0;
    const size_t nr = p.roots.size();
    size_t i = 0;
    auto pick_outer = [&](const void* a, const void* b) -> void* {
        for (void* buf : ch.pool)
            if (buf != a && buf != b) return buf;
        fail(PPA_ERR_INVALID, "internal: apply buffer pool exhausted");
    };
    while (i < nr) {
        const cplx eta = p.roots[i];
        const bool pair = eta.imag() != 0.0;
        const bool last = (i + (pair ? 2 : 1)) >= nr;
        if (!pair) {
            void* out = last ? y : pick_outer(w, v0);
            const VecT ot = last ? vout : chain;
            pi_chain(ch, p.roots1, w, 1.0 / eta.real(), 1.0 - 1.0 / eta.real(), w, 0.0, nullptr, out,
                     ot, {w, v0});
            w = out;
            i += 1;
        } else {
            const double a = eta.real();
            const double q = eta.real() * eta.real() + eta.imag() * eta.imag();
            void* sb = pick_outer(w, v0);
            pi_chain(ch, p.roots1, w, 1.0, 2.0 * a - 1.0, w, 0.0, nullptr, sb, chain, {w, v0});
            void* out = nullptr;
            if (last) {
                out = y;
            } else {
                for (void* buf : ch.pool)
                    if (buf != w && buf != v0 && buf != sb) { out = buf; break; }
                PPA_REQUIRE(out != nullptr, "internal: apply buffer pool exhausted");
            }
            pi_chain(ch, p.roots1, sb, 1.0 / q, 1.0, w, -1.0 / q, sb, out, last ? vout : chain,
                     {w, v0, sb});
            w = out;
            i += 2;
        }
    }
}

}  // namespace

size_t apply_poly(const Matrix& A, const Poly& p, VecT vin, const void* v, VecT vout, void* y,
                  VecT chain, ApplyWs& ws, hipStream_t s) {
    PPA_REQUIRE(p.degree() >= 1, "apply: empty polynomial");
    Chain ch{A, chain, s, {}};
    ch.sigma = p.shift;
    const int nb = apply_buffers(p);
    for (int i = 0; i < nb; ++i) ch.pool.push_back(ws.buf[i]);
    const void* v0 = v;
    if (vin != chain) {
        // bring the input into the chain precision (one streaming pass)
        void* cv = ch.pool.back();
        ch.pool.pop_back();
        if (chain == VecT::F32)
            launch_cast_f64_f32((const double*)v, (float*)cv, A.n, s);
        else
            launch_cast_f32_f64((const float*)v, (double*)cv, A.n, s);
        v0 = cv;
    }
    run_apply(ch, p, v0, vout, y);
    return ch.bytes;
}

size_t apply_poly_bytes(const Matrix& A, const Poly& p, VecT chain) {
    PPA_REQUIRE(p.degree() >= 1, "apply: empty polynomial");
    Chain ch{A, chain, nullptr, {}};
    ch.dry = true;
    ch.sigma = p.shift;
    // stand-in addresses: only their identity matters for the count
    static char tags[10];
    const int nb = apply_buffers(p);
    for (int i = 0; i < nb; ++i) ch.pool.push_back(&tags[i]);
    run_apply(ch, p, &tags[8], chain, &tags[9]);
    return ch.bytes;
}

// ---------------------------------------------------------------- stability
// Section 7.  pof(j) = prod_{i != j} |1 - theta_j / theta_i| is the product of
// the other factors of pi at theta_j (|pi'(theta_j)| = pof(j) / |theta_j|); a
// large value means the factored product amplifies the component along an
// eigenvector near theta_j and cancels it again in one factor.  It is formed
// as a sum of base-10 logarithms so that high degrees do not overflow.
std::vector<double> log10_pof(const std::vector<cplx>& th) {
    const size_t d = th.size();
    std::vector<double> out(d, 0.0);
    for (size_t j = 0; j < d; ++j) {
        double acc = 0.0;
        for (size_t i = 0; i < d; ++i) {
            if (i == j) continue;
            acc += std::log10(std::abs(1.0 - th[j] / th[i]));   // -inf for a repeated root
        }
        out[j] = acc;
    }
    return out;
}

// One extra copy of theta_j for every factor 1e14 by which pof(j) exceeds
// 1e4: ceil((log10 pof(j) - 4) / 14), never negative.
std::vector<int> extra_root_counts(const std::vector<cplx>& th) {
    const std::vector<double> lp = log10_pof(th);
    std::vector<int> c(th.size(), 0);
    for (size_t j = 0; j < th.size(); ++j) {
        const double x = std::ceil((lp[j] - 4.0) / 14.0);
        c[j] = (std::isfinite(x) && x > 0.0) ? (int)x : 0;
    }
    return c;
}

// The extra copies placed as section 7 describes, in list order (a
// conjugate pair is one unit, handled at its Im > 0 member): the first copy
// is appended to the current list; the remaining c - 1 go to positions
// p + round(k (L - p) / c), k = 1..c-1, between the root's position p and
// the end of the list as it stood before this root's copies (length L),
// moved past the second member when a position falls inside a pair.
std::vector<cplx> add_stability_roots(const std::vector<cplx>& th, int* added) {
    const std::vector<int> cnt = extra_root_counts(th);
    std::vector<cplx> out = th;
    int total = 0;
    for (size_t j = 0; j < th.size(); ++j) {
        const int c = cnt[j];
        const cplx z = th[j];
        if (c == 0 || z.imag() < 0.0) continue;
        std::vector<cplx> unit{z};
        if (z.imag() > 0.0) unit.push_back(std::conj(z));
        size_t p = 0;
        while (out[p] != z) ++p;
        const size_t L = out.size();
        std::vector<size_t> spots;
        for (int k = 1; k < c; ++k) {
            size_t q = p + (size_t)std::floor((double)k * (double)(L - p) / (double)c + 0.5);
            if (q > 0 && q < out.size() && out[q - 1].imag() > 0.0 && out[q] == std::conj(out[q - 1]))
                ++q;
            spots.push_back(q);
        }
        out.insert(out.end(), unit.begin(), unit.end());
        std::sort(spots.begin(), spots.end());
        for (auto it = spots.rbegin(); it != spots.rend(); ++it)
            out.insert(out.begin() + (std::ptrdiff_t)*it, unit.begin(), unit.end());
        total += c * (int)unit.size();
    }
    if (added) *added = total;
    return out;
}

}  // namespace ppa
