// Host planning of the projected problem of a restart cycle (section 2 step
// 2, section 4): Ritz pairs of H_m ordered by |target - nu|, the wanted Ritz
// vectors as real columns, Rayleigh quotients and residuals from device dot
// products, and the thick-restart basis change.  Shared by the single-solve
// driver and the batched small-solve engine.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "ppa_internal.hpp"

namespace ppa {

std::vector<int> sort_ritz(const std::vector<cplx>& nu, double target) {
    std::vector<int> idx(nu.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        const double da = std::abs(target - nu[a]), db = std::abs(target - nu[b]);
        if (da != db) return da < db;
        if (nu[a].imag() != nu[b].imag()) return nu[a].imag() > nu[b].imag();
        return nu[a].real() < nu[b].real();
    });
    return idx;
}

RitzPlan plan_ritz(const std::vector<double>& Hm, int mc, int nev, double target, bool harmonic,
                   double hm) {
    RitzPlan R;
    R.mc = mc;
    std::vector<cplx> nu0, G0;
    if (harmonic && hm != 0.0) {
        // harmonic Ritz pairs: (H_m - tau I)^T f = e_m, eig(H_m + hm^2 f e_m^T)
        std::vector<double> T((size_t)mc * mc);
        for (int j = 0; j < mc; ++j)
            for (int i = 0; i < mc; ++i)
                T[i + (size_t)j * mc] = Hm[j + (size_t)i * mc] - (i == j ? target : 0.0);
        std::vector<double> f(mc, 0.0);
        f[mc - 1] = 1.0;
        if (lu_solve(mc, T, f)) {
            std::vector<double> M = Hm;
            for (int i = 0; i < mc; ++i) M[i + (size_t)(mc - 1) * mc] += hm * hm * f[i];
            dense_eig(mc, M.data(), nu0, &G0);
            R.harmonic = true;
            R.fh = f;
            R.hm = hm;
        }
    }
    if (!R.harmonic) dense_eig(mc, Hm.data(), nu0, &G0);
    const std::vector<int> ord = sort_ritz(nu0, target);
    R.nu.resize(mc);
    R.G.resize((size_t)mc * mc);
    for (int i = 0; i < mc; ++i) {
        R.nu[i] = nu0[ord[i]];
        for (int q = 0; q < mc; ++q) R.G[q + (size_t)i * mc] = G0[q + (size_t)ord[i] * mc];
    }
    R.nw = std::min(nev, mc);
    for (int i = 0; i < R.nw; ++i) {
        const cplx* g = &R.G[(size_t)i * mc];
        if (R.nu[i].imag() == 0.0) {
            R.cre.push_back(R.ycols);
            R.cim.push_back(-1);
            R.dup.push_back(0);
            for (int q = 0; q < mc; ++q) R.Gw.push_back(g[q].real());
            R.ycols += 1;
        } else if (R.nu[i].imag() > 0.0 || i == 0 || R.nu[i - 1] != std::conj(R.nu[i])) {
            // y = V g held as two real columns, Re g and Im g
            R.cre.push_back(R.ycols);
            R.cim.push_back(R.ycols + 1);
            R.dup.push_back(0);
            for (int q = 0; q < mc; ++q) R.Gw.push_back(g[q].real());
            for (int q = 0; q < mc; ++q) R.Gw.push_back(g[q].imag());
            R.ycols += 2;
        } else {
            // conjugate of the previous wanted value: same columns
            R.cre.push_back(R.cre.back());
            R.cim.push_back(R.cim.back());
            R.dup.push_back(1);
        }
    }
    return R;
}

std::vector<DotSpec> ritz_dots(const RitzPlan& R) {
    std::vector<DotSpec> d;
    for (int i = 0; i < R.nw; ++i) {
        if (R.dup[i]) continue;
        const int a = R.cre[i], b = R.cim[i];
        d.push_back({a, a, 1});   // y_a . y_a
        d.push_back({a, a, 0});   // y_a . (A y)_a
        if (b >= 0) {
            d.push_back({b, b, 1});
            d.push_back({b, b, 0});
            d.push_back({a, b, 0});   // y_a . (A y)_b
            d.push_back({b, a, 0});   // y_b . (A y)_a
        }
    }
    return d;
}

void ritz_mu(const RitzPlan& R, const std::vector<double>& dv, std::vector<cplx>& mu,
             std::vector<double>& ynorm) {
    mu.assign(R.nw, cplx(0.0, 0.0));
    ynorm.assign(R.nw, 0.0);
    size_t t = 0;
    for (int i = 0; i < R.nw; ++i) {
        if (R.dup[i]) {
            mu[i] = std::conj(mu[i - 1]);
            ynorm[i] = ynorm[i - 1];
            continue;
        }
        if (R.cim[i] < 0) {
            const double yy = dv[t], yAy = dv[t + 1];
            t += 2;
            mu[i] = cplx(yAy / yy, 0.0);
            ynorm[i] = std::sqrt(yy);
        } else {
            // y = a + i b: y^* y = a.a + b.b,
            // y^* A y = a.Aa + b.Ab + i (a.Ab - b.Aa)
            const double aa = dv[t], aAa = dv[t + 1], bb = dv[t + 2], bAb = dv[t + 3];
            const double aAb = dv[t + 4], bAa = dv[t + 5];
            t += 6;
            const double yy = aa + bb;
            mu[i] = cplx(aAa + bAb, aAb - bAa) / yy;
            ynorm[i] = std::sqrt(yy);
        }
    }
}

std::vector<ComboSpec> ritz_combos(const RitzPlan& R, const std::vector<cplx>& mu) {
    std::vector<ComboSpec> L;
    for (int i = 0; i < R.nw; ++i) {
        if (R.dup[i]) continue;
        const int a = R.cre[i], b = R.cim[i];
        const double mr = mu[i].real(), mi = mu[i].imag();
        if (b < 0) {
            L.push_back({i, {a, a, -1}, {0, 1, 1}, {1.0, -mr, 0.0}, 2});
        } else {
            // A y - mu y with y = a + i b, mu = mr + i mi:
            // real part A a - mr a + mi b, imaginary part A b - mr b - mi a
            L.push_back({i, {a, a, b}, {0, 1, 1}, {1.0, -mr, mi}, 3});
            L.push_back({i, {b, b, a}, {0, 1, 1}, {1.0, -mr, -mi}, 3});
        }
    }
    return L;
}

void ritz_resid(const RitzPlan& R, const std::vector<ComboSpec>& cs, const std::vector<double>& rn,
                const std::vector<double>& ynorm, std::vector<double>& res) {
    std::vector<double> acc(R.nw, 0.0);
    for (size_t q = 0; q < cs.size(); ++q) acc[cs[q].owner] += rn[q];
    res.assign(R.nw, 0.0);
    for (int i = 0; i < R.nw; ++i)
        res[i] = R.dup[i] ? res[i - 1] : std::sqrt(acc[i]) / ynorm[i];
}

int64_t ritz_mvps(const RitzPlan& R) {
    int64_t m = 0;
    for (int i = 0; i < R.nw; ++i) m += (R.nu[i].imag() == 0.0) ? 1 : 2;
    return m;
}

bool leave_fp32(const std::vector<double>& hist, double anorm) {
    const size_t hc = hist.size();
    if (hc == 0) return false;
    const double mx = hist[hc - 1];
    const double floor_abs = 100.0 * 1.1920929e-07 * anorm;
    const bool floor = mx <= floor_abs;
    const bool stall = hc >= 3 && mx > 0.5 * hist[hc - 3] && mx <= 1e3 * floor_abs;
    return floor || stall;
}

RestartPlan plan_restart(const RitzPlan& R, const std::vector<double>& Hm, double hm, int m, int k) {
    const int mc = R.mc;
    RestartPlan P;
    int kk = std::min(k, mc - 1);
    if (kk < mc && R.nu[kk - 1].imag() > 0.0) kk -= 1;
    if (kk == 0) kk = std::min(2, mc - 1);
    std::vector<double> B;
    for (int i = 0; i < kk; ++i) {
        const cplx* g = &R.G[(size_t)i * mc];
        if (R.nu[i].imag() == 0.0) {
            for (int q = 0; q < mc; ++q) B.push_back(g[q].real());
        } else if (R.nu[i].imag() > 0.0) {
            for (int q = 0; q < mc; ++q) B.push_back(g[q].real());
            for (int q = 0; q < mc; ++q) B.push_back(g[q].imag());
        }
    }
    P.kk = kk;
    orthonormal_basis(mc, kk, B, P.Q);
    // Q' = [[Q, 0], [0, 1]]  ((m+1) x (kk+1)): [V_m Q, v_{m+1}]
    P.Qp.assign((size_t)(m + 1) * (kk + 1), 0.0);
    for (int jj = 0; jj < kk; ++jj)
        for (int i = 0; i < mc; ++i) P.Qp[i + (size_t)jj * (m + 1)] = P.Q[i + (size_t)jj * mc];
    P.Qp[m + (size_t)kk * (m + 1)] = 1.0;
    // H_k = Q^T H_m Q and the spike row h_{m+1,m} e_m^T Q
    std::vector<double> HQ((size_t)mc * kk, 0.0);
    P.Hn.assign((size_t)(m + 1) * m, 0.0);
    for (int jj = 0; jj < kk; ++jj)
        for (int i = 0; i < mc; ++i) {
            double s = 0.0;
            for (int q = 0; q < mc; ++q) s += Hm[i + (size_t)q * mc] * P.Q[q + (size_t)jj * mc];
            HQ[i + (size_t)jj * mc] = s;
        }
    for (int jj = 0; jj < kk; ++jj)
        for (int i = 0; i < kk; ++i) {
            double s = 0.0;
            for (int q = 0; q < mc; ++q) s += P.Q[q + (size_t)i * mc] * HQ[q + (size_t)jj * mc];
            P.Hn[i + (size_t)jj * (m + 1)] = s;
        }
    for (int jj = 0; jj < kk; ++jj) P.Hn[kk + (size_t)jj * (m + 1)] = hm * P.Q[(mc - 1) + (size_t)jj * mc];
    if (!R.harmonic || mc != m) return P;
    // Harmonic restart: every kept harmonic Ritz pair's residual is parallel
    // to v_{m+1} - hm V_m f, so the next basis vector is [-hm f; 1]
    // orthonormalised against [Q; 0] (twice), and the new projected block is
    // [Q; 0 | w]^T Hbar_m Q, a full (kk+1) x kk matrix.
    std::vector<double> w(m + 1, 0.0);
    for (int i = 0; i < m; ++i) w[i] = -hm * R.fh[i];
    w[m] = 1.0;
    for (int pass = 0; pass < 2; ++pass)
        for (int jj = 0; jj < kk; ++jj) {
            double c = 0.0;
            for (int i = 0; i < m; ++i) c += P.Q[i + (size_t)jj * mc] * w[i];
            for (int i = 0; i < m; ++i) w[i] -= c * P.Q[i + (size_t)jj * mc];
        }
    double nw = 0.0;
    for (double x : w) nw += x * x;
    nw = std::sqrt(nw);
    for (int i = 0; i <= m; ++i) P.Qp[i + (size_t)kk * (m + 1)] = w[i] / nw;
    // Hbar Q ((m+1) x kk) with Hbar = [H_m; hm e_m^T]
    std::vector<double> HQ1((size_t)(m + 1) * kk, 0.0);
    for (int jj = 0; jj < kk; ++jj) {
        for (int i = 0; i < m; ++i) HQ1[i + (size_t)jj * (m + 1)] = HQ[i + (size_t)jj * mc];
        HQ1[m + (size_t)jj * (m + 1)] = hm * P.Q[(m - 1) + (size_t)jj * mc];
    }
    for (int jj = 0; jj < kk; ++jj)
        for (int i = 0; i <= kk; ++i) {
            double acc = 0.0;
            for (int r = 0; r <= m; ++r) acc += P.Qp[r + (size_t)i * (m + 1)] * HQ1[r + (size_t)jj * (m + 1)];
            P.Hn[i + (size_t)jj * (m + 1)] = acc;
        }
    return P;
}

}  // namespace ppa
