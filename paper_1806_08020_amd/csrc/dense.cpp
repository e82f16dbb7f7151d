// Small dense real nonsymmetric linear algebra on the host, FP64.
//
// The projected problems of the method are tiny (d x d for the harmonic Ritz
// values of section 2 step 1(b), m x m for the Ritz pairs of each restart
// cycle, m <= 64, d <= a few hundred) and their eigen-decompositions sit
// between device phases, so they run on the host:
//  * Householder reduction to upper Hessenberg form, accumulating Q;
//  * Francis implicit double-shift QR iteration to real Schur form
//    (Golub & Van Loan, Matrix Computations, sections 7.4-7.5), with real 2x2
//    blocks split by a rotation so only complex pairs remain as 2x2 blocks;
//  * eigenvectors of the quasi-triangular factor by back substitution in
//    complex arithmetic, mapped back with the accumulated Schur vectors;
//  * Gaussian elimination with partial pivoting and Householder QR.
// All matrices are column-major: a(i, j) = a[i + j * n].
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>

#include "ppa_internal.hpp"

namespace ppa {

namespace {

struct Mat {
    int n, m;
    std::vector<double> a;
    Mat(int rows, int cols) : n(rows), m(cols), a((size_t)rows * cols, 0.0) {}
    double& operator()(int i, int j) { return a[i + (size_t)j * n]; }
    double operator()(int i, int j) const { return a[i + (size_t)j * n]; }
};

// Householder vector for x (length len): v[0] = 1, returns beta with
// (I - beta v v^T) x = alpha e_1; beta = 0 when x is already a multiple of e_1.
double householder(const double* x, int len, double* v, double* alpha_out) {
    double s = 0.0;
    for (int i = 1; i < len; ++i) s += x[i] * x[i];
    v[0] = 1.0;
    if (s == 0.0) {
        for (int i = 1; i < len; ++i) v[i] = 0.0;
        *alpha_out = x[0];
        return 0.0;
    }
    const double nrm = std::sqrt(x[0] * x[0] + s);
    const double alpha = x[0] >= 0.0 ? -nrm : nrm;
    const double u0 = x[0] - alpha;
    for (int i = 1; i < len; ++i) v[i] = x[i] / u0;
    *alpha_out = alpha;
    return -u0 / alpha;   // = 2 / (v^T v)
}

void hessenberg_reduce(Mat& A, Mat& Q) {
    const int n = A.n;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Q(i, j) = (i == j) ? 1.0 : 0.0;
    std::vector<double> x(n), v(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int len = n - k - 1;
        for (int i = 0; i < len; ++i) x[i] = A(k + 1 + i, k);
        double alpha;
        const double beta = householder(x.data(), len, v.data(), &alpha);
        if (beta == 0.0) continue;
        // left: rows k+1.., columns k..n-1
        for (int j = k; j < n; ++j) {
            double s = 0.0;
            for (int i = 0; i < len; ++i) s += v[i] * A(k + 1 + i, j);
            s *= beta;
            for (int i = 0; i < len; ++i) A(k + 1 + i, j) -= s * v[i];
        }
        // right: all rows, columns k+1..
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int t = 0; t < len; ++t) s += A(i, k + 1 + t) * v[t];
            s *= beta;
            for (int t = 0; t < len; ++t) A(i, k + 1 + t) -= s * v[t];
        }
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int t = 0; t < len; ++t) s += Q(i, k + 1 + t) * v[t];
            s *= beta;
            for (int t = 0; t < len; ++t) Q(i, k + 1 + t) -= s * v[t];
        }
        A(k + 1, k) = alpha;
        for (int i = k + 2; i < n; ++i) A(i, k) = 0.0;
    }
}

// Apply the reflector (I - beta v v^T), v = (1, v1[, v2]), of size `len`
// acting on indices p.. of H's rows (columns c0..c1) and columns (rows r0..r1),
// and on Z's columns.
void reflect_rows(Mat& H, int p, int len, const double* v, double beta, int c0, int c1) {
    for (int j = c0; j <= c1; ++j) {
        double s = 0.0;
        for (int t = 0; t < len; ++t) s += v[t] * H(p + t, j);
        s *= beta;
        for (int t = 0; t < len; ++t) H(p + t, j) -= s * v[t];
    }
}
void reflect_cols(Mat& H, int p, int len, const double* v, double beta, int r0, int r1) {
    for (int i = r0; i <= r1; ++i) {
        double s = 0.0;
        for (int t = 0; t < len; ++t) s += H(i, p + t) * v[t];
        s *= beta;
        for (int t = 0; t < len; ++t) H(i, p + t) -= s * v[t];
    }
}

// Rotation G = [cs -sn; sn cs] applied as H <- G^T H G on indices (p, p+1).
void rotate(Mat& H, Mat* Z, int p, double cs, double sn) {
    const int n = H.n;
    for (int j = p; j < n; ++j) {
        const double a = H(p, j), b = H(p + 1, j);
        H(p, j) = cs * a + sn * b;
        H(p + 1, j) = -sn * a + cs * b;
    }
    for (int i = 0; i <= std::min(p + 1, n - 1); ++i) {
        const double a = H(i, p), b = H(i, p + 1);
        H(i, p) = cs * a + sn * b;
        H(i, p + 1) = -sn * a + cs * b;
    }
    if (Z) {
        for (int i = 0; i < Z->n; ++i) {
            const double a = (*Z)(i, p), b = (*Z)(i, p + 1);
            (*Z)(i, p) = cs * a + sn * b;
            (*Z)(i, p + 1) = -sn * a + cs * b;
        }
    }
}

// Francis double-shift QR on an upper Hessenberg H (full Schur form, all
// columns / rows updated), accumulating into Z when non-null.  On success H is
// quasi-upper-triangular with 2x2 blocks only for complex conjugate pairs.
bool schur(Mat& H, Mat* Z, std::vector<cplx>& w) {
    const int n = H.n;
    w.assign(n, cplx(0.0, 0.0));
    if (n == 0) return true;
    double anorm = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= std::min(j + 1, n - 1); ++i) anorm += std::fabs(H(i, j));
    const double eps = DBL_EPSILON;
    const double smlnum = DBL_MIN * ((double)n / eps);
    const int itmax = 30 * std::max(10, n);
    int hi = n - 1, its = 0, total = 0;
    double v[3];
    while (hi >= 0) {
        int l = hi;
        for (; l > 0; --l) {
            double s = std::fabs(H(l - 1, l - 1)) + std::fabs(H(l, l));
            if (s == 0.0) s = anorm;
            if (std::fabs(H(l, l - 1)) <= smlnum || std::fabs(H(l, l - 1)) <= eps * s) {
                H(l, l - 1) = 0.0;
                break;
            }
        }
        if (l == hi) {
            w[hi] = cplx(H(hi, hi), 0.0);
            --hi;
            its = 0;
            continue;
        }
        if (l == hi - 1) {
            const int p = hi - 1;
            const double a = H(p, p), b = H(p, p + 1), c = H(p + 1, p), d = H(p + 1, p + 1);
            const double pp = 0.5 * (a - d);
            const double disc = pp * pp + b * c;
            if (disc >= 0.0) {
                // real pair: rotate the block to upper triangular form
                const double z = pp + (pp >= 0.0 ? std::sqrt(disc) : -std::sqrt(disc));
                const double lam = d + z;
                double e0 = b, e1 = lam - a;
                if (std::fabs(b) + std::fabs(lam - a) < std::fabs(lam - d) + std::fabs(c)) {
                    e0 = lam - d;
                    e1 = c;
                }
                const double r = std::hypot(e0, e1);
                if (r > 0.0) rotate(H, Z, p, e0 / r, e1 / r);
                H(p + 1, p) = 0.0;
                w[p] = cplx(H(p, p), 0.0);
                w[p + 1] = cplx(H(p + 1, p + 1), 0.0);
            } else {
                const double re = 0.5 * (a + d), im = std::sqrt(-disc);
                w[p] = cplx(re, im);
                w[p + 1] = cplx(re, -im);
            }
            hi -= 2;
            its = 0;
            continue;
        }
        if (total >= itmax) return false;
        // the shift pair: a complex pair re +- i im (im > 0), or one real
        // shift re used twice (im = 0)
        double re, im;
        if (its > 0 && its % 10 == 0) {
            // exceptional shifts (a conjugate pair) from the trailing or, every
            // other time, the leading corner of the active window
            const bool top = (its / 10) % 2 == 0;
            const double ex = top ? std::fabs(H(l + 1, l)) + std::fabs(H(l + 2, l + 1))
                                  : std::fabs(H(hi, hi - 1)) + std::fabs(H(hi - 1, hi - 2));
            const double base = top ? H(l, l) : H(hi, hi);
            re = base + 0.75 * ex;
            im = 0.66 * ex;
        } else {
            // eigenvalues of the trailing 2 x 2 block; two real ones are
            // replaced by the one nearer H(hi, hi), taken twice
            const double a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
            const double pp = 0.5 * (a - d), disc = pp * pp + b * c;
            const double mid = 0.5 * (a + d);
            if (disc >= 0.0) {
                const double sq = std::sqrt(disc);
                const double r1 = mid + sq, r2 = mid - sq;
                re = std::fabs(r1 - d) <= std::fabs(r2 - d) ? r1 : r2;
                im = 0.0;
            } else {
                re = mid;
                im = std::sqrt(-disc);
            }
        }
        ++its;
        ++total;
        // first column of (H - sigma1)(H - sigma2) restricted to rows l, l+1,
        // l+2, formed from the differences H(l, l) - re (no cancellation when
        // the shifts are close to H(l, l), as for a multiple eigenvalue) and
        // scaled by sc: only its direction matters
        const double h21 = H(l + 1, l);
        double sc = std::fabs(H(l, l) - re) + im + std::fabs(h21);
        if (sc == 0.0) sc = 1.0;
        const double h21s = h21 / sc, d11 = H(l, l) - re;
        double x = h21s * H(l, l + 1) + d11 * (d11 / sc) + im * (im / sc);
        double y = h21s * (d11 + (H(l + 1, l + 1) - re));
        double z = h21s * H(l + 2, l + 1);
        for (int k = l; k <= hi - 2; ++k) {
            const double xv[3] = {x, y, z};
            double alpha;
            const double beta = householder(xv, 3, v, &alpha);
            if (beta != 0.0) {
                const int q = std::max(l, k - 1);
                reflect_rows(H, k, 3, v, beta, q, n - 1);
                reflect_cols(H, k, 3, v, beta, 0, std::min(k + 3, hi));
                if (Z) reflect_cols(*Z, k, 3, v, beta, 0, Z->n - 1);
                if (k > l) {
                    H(k, k - 1) = alpha;
                    H(k + 1, k - 1) = 0.0;
                    H(k + 2, k - 1) = 0.0;
                }
            }
            x = H(k + 1, k);
            y = H(k + 2, k);
            if (k < hi - 2) z = H(k + 3, k);
        }
        {
            const double xv[2] = {x, y};
            double alpha;
            const double beta = householder(xv, 2, v, &alpha);
            if (beta != 0.0) {
                reflect_rows(H, hi - 1, 2, v, beta, std::max(l, hi - 2), n - 1);
                reflect_cols(H, hi - 1, 2, v, beta, 0, hi);
                if (Z) reflect_cols(*Z, hi - 1, 2, v, beta, 0, Z->n - 1);
                if (hi - 2 >= l) {
                    H(hi - 1, hi - 2) = alpha;
                    H(hi, hi - 2) = 0.0;
                }
            }
        }
    }
    return true;
}

// Eigenvector of the quasi-triangular T for eigenvalue w[p] (p = first row of
// its block), by back substitution in complex arithmetic.
void tri_eigvec(const Mat& T, const std::vector<cplx>& w, int p, double smin, std::vector<cplx>& x) {
    const int n = T.n;
    x.assign(n, cplx(0.0, 0.0));
    const cplx lam = w[p];
    int top, last;
    const bool block = (p + 1 < n) && T(p + 1, p) != 0.0;
    if (!block) {
        x[p] = 1.0;
        top = p - 1;
        last = p;
    } else {
        cplx den = T(p, p) - lam;
        if (std::abs(den) < smin) den = smin;
        x[p + 1] = 1.0;
        x[p] = -T(p, p + 1) / den;
        top = p - 1;
        last = p + 1;
    }
    for (int i = top; i >= 0;) {
        if (i >= 1 && T(i, i - 1) != 0.0) {
            cplx r1 = 0.0, r2 = 0.0;
            for (int j = i + 1; j <= last; ++j) {
                r1 -= T(i - 1, j) * x[j];
                r2 -= T(i, j) * x[j];
            }
            const cplx a = T(i - 1, i - 1) - lam, b = T(i - 1, i), c = T(i, i - 1), d = T(i, i) - lam;
            cplx det = a * d - b * c;
            if (std::abs(det) < smin * smin) det = smin * smin;
            x[i - 1] = (r1 * d - b * r2) / det;
            x[i] = (a * r2 - c * r1) / det;
            i -= 2;
        } else {
            cplx r = 0.0;
            for (int j = i + 1; j <= last; ++j) r -= T(i, j) * x[j];
            cplx den = T(i, i) - lam;
            if (std::abs(den) < smin) den = smin;
            x[i] = r / den;
            i -= 1;
        }
        double mx = 0.0;
        for (int j = 0; j <= last; ++j) mx = std::max(mx, std::abs(x[j]));
        if (mx > 1e150)
            for (int j = 0; j <= last; ++j) x[j] /= mx;
    }
}

}  // namespace

// One attempt: Hessenberg reduction, Francis QR, eigenvectors.  (No diagonal
// balancing: after a thick restart H_m is nearly block triangular, and the
// large scalings balancing would pick make the mapped-back eigenvectors
// inaccurate in norm, which is the accuracy the restart needs.)
static bool eig_attempt(int n, const Mat& A0, std::vector<cplx>& w, std::vector<cplx>* V) {
    Mat H = A0, Q(n, n);
    hessenberg_reduce(H, Q);
    if (!schur(H, V ? &Q : nullptr, w)) return false;
    if (!V) return true;
    double tn = 0.0;
    for (double e : H.a) tn = std::max(tn, std::fabs(e));
    const double smin = std::max(DBL_EPSILON * tn, DBL_MIN);
    V->assign((size_t)n * n, cplx(0.0, 0.0));
    std::vector<cplx> x;
    for (int p = 0; p < n; ++p) {
        if (w[p].imag() < 0.0) {
            // conjugate of the previous column
            for (int i = 0; i < n; ++i) (*V)[i + (size_t)p * n] = std::conj((*V)[i + (size_t)(p - 1) * n]);
            continue;
        }
        tri_eigvec(H, w, p, smin, x);
        double nrm = 0.0;
        for (int i = 0; i < n; ++i) {
            cplx s = 0.0;
            for (int j = 0; j < n; ++j) s += Q(i, j) * x[j];
            (*V)[i + (size_t)p * n] = s;
            nrm += std::norm(s);
        }
        nrm = std::sqrt(nrm);
        if (nrm > 0.0)
            for (int i = 0; i < n; ++i) (*V)[i + (size_t)p * n] /= nrm;
    }
    return true;
}

void dense_eig(int n, const double* a, std::vector<cplx>& w, std::vector<cplx>* V) {
    Mat A(n, n);
    std::copy(a, a + (size_t)n * n, A.a.begin());
    for (double e : A.a)
        if (!std::isfinite(e)) fail(PPA_ERR_NONFINITE, "dense_eig: non-finite matrix entry");
    if (eig_attempt(n, A, w, V)) return;
    // Rare stagnation of the shifted QR: retry on orthogonally similar
    // matrices Z^T A Z (same eigenvalues; eigenvectors mapped back by Z).
    for (int attempt = 1; attempt <= 3; ++attempt) {
        Mat Z(n, n), B(n, n), T(n, n);
        uint64_t state = 0x9E3779B97F4A7C15ull * (uint64_t)attempt + (uint64_t)n;
        for (double& e : Z.a) {
            state ^= state << 13; state ^= state >> 7; state ^= state << 17;
            e = (double)(state >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        }
        std::vector<double> Zq;
        orthonormal_basis(n, n, Z.a, Zq);
        Z.a = Zq;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double t = 0.0;
                for (int k = 0; k < n; ++k) t += A(i, k) * Z(k, j);
                T(i, j) = t;
            }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double t = 0.0;
                for (int k = 0; k < n; ++k) t += Z(k, i) * T(k, j);
                B(i, j) = t;
            }
        std::vector<cplx> Vb;
        if (!eig_attempt(n, B, w, V ? &Vb : nullptr)) continue;
        if (V) {
            V->assign((size_t)n * n, cplx(0.0, 0.0));
            for (int p = 0; p < n; ++p)
                for (int i = 0; i < n; ++i) {
                    cplx s = 0.0;
                    for (int k = 0; k < n; ++k) s += Z(i, k) * Vb[k + (size_t)p * n];
                    (*V)[i + (size_t)p * n] = s;
                }
        }
        return;
    }
    fail(PPA_ERR_NUMERIC, "dense_eig: QR iteration did not converge (n=%d)", n);
}

void hessenberg_eigvals(int n, std::vector<double>& h, std::vector<cplx>& w) {
    Mat H(n, n);
    H.a = h;
    if (schur(H, nullptr, w)) return;
    // fall back to the general path (retries on similar matrices)
    dense_eig(n, h.data(), w, nullptr);
}

bool lu_solve(int n, std::vector<double> M, std::vector<double>& b) {
    auto at = [&](int i, int j) -> double& { return M[i + (size_t)j * n]; };
    double mx = 0.0;
    for (double e : M) mx = std::max(mx, std::fabs(e));
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(at(i, k)) > std::fabs(at(piv, k))) piv = i;
        if (!(std::fabs(at(piv, k)) > mx * DBL_EPSILON * 4)) return false;
        if (piv != k) {
            for (int j = 0; j < n; ++j) std::swap(at(k, j), at(piv, j));
            std::swap(b[k], b[piv]);
        }
        for (int i = k + 1; i < n; ++i) {
            const double f = at(i, k) / at(k, k);
            if (f == 0.0) continue;
            for (int j = k + 1; j < n; ++j) at(i, j) -= f * at(k, j);
            b[i] -= f * b[k];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < n; ++j) s -= at(i, j) * b[j];
        b[i] = s / at(i, i);
    }
    return true;
}

void orthonormal_basis(int m, int k, const std::vector<double>& B, std::vector<double>& Q) {
    // Householder QR of B (m x k), then Q = H_1 ... H_k [I_k; 0]
    std::vector<double> R = B;
    std::vector<std::vector<double>> vs(k);
    std::vector<double> betas(k);
    std::vector<double> x(m), v(m);
    for (int j = 0; j < k; ++j) {
        const int len = m - j;
        for (int i = 0; i < len; ++i) x[i] = R[(j + i) + (size_t)j * m];
        double alpha;
        betas[j] = householder(x.data(), len, v.data(), &alpha);
        vs[j].assign(v.begin(), v.begin() + len);
        for (int c = j; c < k; ++c) {
            double s = 0.0;
            for (int i = 0; i < len; ++i) s += v[i] * R[(j + i) + (size_t)c * m];
            s *= betas[j];
            for (int i = 0; i < len; ++i) R[(j + i) + (size_t)c * m] -= s * v[i];
        }
    }
    Q.assign((size_t)m * k, 0.0);
    for (int j = 0; j < k; ++j) Q[j + (size_t)j * m] = 1.0;
    for (int j = k - 1; j >= 0; --j) {
        const int len = m - j;
        for (int c = 0; c < k; ++c) {
            double s = 0.0;
            for (int i = 0; i < len; ++i) s += vs[j][i] * Q[(j + i) + (size_t)c * m];
            s *= betas[j];
            for (int i = 0; i < len; ++i) Q[(j + i) + (size_t)c * m] -= s * vs[j][i];
        }
    }
}

}  // namespace ppa
