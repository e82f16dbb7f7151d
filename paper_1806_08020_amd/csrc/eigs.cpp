// GMRES polynomial construction on the device (section 2, step 1; section 8)
// and thick-restarted Arnoldi(m,k) on pi(A) (section 2 step 2, section 4).
//
// Device work per Krylov step: one application of the polynomial operator
// (d fused SpMV passes) and one CGS2 orthogonalisation.  The host sees the
// small projected matrix once per cycle (one stream synchronisation), solves
// the m x m eigenproblem, and drives the Ritz test and the restart, whose
// n-sized work (V Q on MFMA, A Y, dots and residual norms) stays on the device.
#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>

#include "ppa_internal.hpp"

namespace ppa {

namespace {

constexpr double kBreakdownTol = 1e-14;

__global__ void k_scale_host(double* v, int64_t n, double s) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v[i] *= s;
}
__global__ void k_copy(const double* __restrict__ in, double* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

unsigned sgrid(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
}

// ||v||^2 of one device vector (deterministic), returned to the host.
double norm2_host(int64_t n, const double* v, double* partial, int nb, double* out_d,
                  hipStream_t s) {
    DotList L{};
    L.a[0] = v;
    L.b[0] = v;
    L.count = 1;
    launch_dots(n, L, partial, nb, out_d, s);
    double r = 0.0;
    PPA_HIP(hipMemcpyAsync(&r, out_d, sizeof(double), hipMemcpyDeviceToHost, s));
    PPA_HIP(hipStreamSynchronize(s));
    return r;
}

// Copy v into dst and normalise it; returns ||v||.
double set_unit(int64_t n, const double* v, double* dst, double* partial, int nb, double* out_d,
                hipStream_t s) {
    const double nn = std::sqrt(norm2_host(n, v, partial, nb, out_d, s));
    if (!(nn > 0.0) || !std::isfinite(nn)) fail(PPA_ERR_NONFINITE, "start vector has zero or non-finite norm");
    if (v != dst) {
        hipLaunchKernelGGL(k_copy, dim3(sgrid(n)), dim3(256), 0, s, v, dst, n);
        PPA_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_scale_host, dim3(sgrid(n)), dim3(256), 0, s, dst, n, 1.0 / nn);
    PPA_HIP(hipGetLastError());
    return nn;
}

// Arnoldi steps j0..m-1 on `op` (op(x, y): y = op x, length N) extending the
// orthonormal basis V (ld) and the Hessenberg matrix Hd (ld ldh, device).
// Default: classical Gram-Schmidt with one reorthogonalisation pass per
// step.  lowsync: the reorthogonalisation delayed by one step (op acts on the
// once-orthogonalised candidate, kept in ub0 / ub1).  mark(j, phase) is
// called before op (0), after op (1) and after the orthogonalisation (2).
// Breakdown is read from H afterwards.
template <class Op, class Mark>
void arnoldi_steps(int64_t N, int j0, int m, bool lowsync, double* V, int64_t ld, double* w,
                   double* Hd, int64_t ldh, double* ub0, double* ub1, Cgs2Ws& cw, hipStream_t s,
                   Op&& op, Mark&& mark, int64_t& dots, int64_t& vops) {
    if (!lowsync) {
        for (int j = j0; j < m; ++j) {
            mark(j, 0);
            op(V + (size_t)j * ld, w);
            mark(j, 1);
            double* vn = V + (size_t)(j + 1) * ld;
            launch_cgs2(N, j + 1, V, ld, w, vn, Hd + (size_t)j * ldh, vn, kBreakdownTol, cw, s);
            mark(j, 2);
            dots += 2 * (j + 1) + 1;
            vops += 4 * (j + 1) + 2;
        }
        return;
    }
    double* ub[2] = {ub0, ub1};
    int cur = 0;
    for (int j = j0; j < m; ++j) {
        mark(j, 0);
        op(j == j0 ? V + (size_t)j * ld : ub[cur], w);
        mark(j, 1);
        if (j == j0) {
            launch_dcgs_step(DCGS_FIRST, N, j + 1, V, ld, nullptr, w, Hd, ldh, nullptr, ub[cur],
                             kBreakdownTol, cw, s);
            dots += j + 1;
            vops += j + 1;
        } else {
            launch_dcgs_step(DCGS_LAGGED, N, j, V, ld, ub[cur], w, Hd, ldh, V + (size_t)j * ld,
                             ub[1 - cur], kBreakdownTol, cw, s);
            cur = 1 - cur;
            dots += 2 * (j + 1);
            vops += 2 * j + 3;
        }
        if (j == m - 1) {
            launch_dcgs_step(DCGS_LAST, N, m, V, ld, ub[cur], nullptr, Hd, ldh, V + (size_t)m * ld,
                             nullptr, kBreakdownTol, cw, s);
            dots += m + 1;
            vops += m + 1;
        }
        mark(j, 2);
    }
}

// ---------------------------------------------------------------- GMRES
struct GmresWs {
    double* V = nullptr;
    int64_t ld = 0;
    double* w = nullptr;
    double* H = nullptr;
    Cgs2Ws cw;
    ApplyWs aw;
    double* dpart = nullptr;
    double* dout = nullptr;
    double* ub0 = nullptr;   // candidates of the delayed Gram-Schmidt
    double* ub1 = nullptr;
};

void carve_gmres(Carver& c, int64_t n, int d, bool tau, GmresWs& g) {
    g.ld = col_ld(n);
    g.V = c.take<double>((size_t)g.ld * (d + 1));
    g.w = c.take<double>((size_t)n);
    g.ub0 = c.take<double>((size_t)n);
    g.ub1 = c.take<double>((size_t)n);
    g.H = c.take<double>((size_t)(d + 1) * d);
    carve_cgs2(c, n, g.cw);
    if (tau) {
        Poly dummy;
        dummy.roots.assign(1, cplx(1.0, 0.0));
        carve_apply(c, n, dummy, VecT::F64, g.aw);
    }
    g.dpart = c.take<double>((size_t)MAX_DOTS * cgs_blocks(n));
    g.dout = c.take<double>(MAX_DOTS);
}

// tau(A) x = x - pi_1(A) x  (F64): the last pass of the pi_1 chain is scaled
// by -1 and adds x in its epilogue.
void apply_tau(const Matrix& A, const std::vector<cplx>& roots1, const double* x, double* out,
               ApplyWs& aw, hipStream_t s, double sigma) {
    apply_single_epilogue(A, roots1, x, out, -1.0, 1.0, x, aw, s, sigma);
}

// One cycle of GMRES(d) from b with operator A (roots1 empty) or tau(A).
// With b2 (section 5, two start vectors; roots1 empty) the cycle runs on the
// block-diagonal system diag(A, A) of dimension 2n from [b; b2], each half
// scaled to norm 1/sqrt(2): the Krylov vectors have length 2n and each
// operator application is one fused pass per half.  The workspace must be
// carved for the vector length used.
// Returns the effective degree; Hbar receives (d_eff+1) x d_eff.
int gmres_cycle(const Matrix& A, const std::vector<cplx>& roots1, int d, const double* b,
                const double* b2, double sigma, GmresWs& g, hipStream_t s,
                std::vector<double>& Hbar, bool lowsync = false) {
    const int64_t n = A.n;
    const int64_t N = b2 ? 2 * n : n;
    launch_zero(g.H, (int64_t)(d + 1) * d, s);
    if (b2) {
        const int nbh = cgs_blocks(n);
        const double n1 = std::sqrt(norm2_host(n, b, g.dpart, nbh, g.dout, s));
        const double n2 = std::sqrt(norm2_host(n, b2, g.dpart, nbh, g.dout, s));
        if (!(n1 > 0.0) || !(n2 > 0.0) || !std::isfinite(n1) || !std::isfinite(n2))
            fail(PPA_ERR_NONFINITE, "start vector has zero or non-finite norm");
        hipLaunchKernelGGL(k_copy, dim3(sgrid(n)), dim3(256), 0, s, b, g.V, n);
        hipLaunchKernelGGL(k_copy, dim3(sgrid(n)), dim3(256), 0, s, b2, g.V + n, n);
        hipLaunchKernelGGL(k_scale_host, dim3(sgrid(n)), dim3(256), 0, s, g.V, n, 1.0 / (std::sqrt(2.0) * n1));
        hipLaunchKernelGGL(k_scale_host, dim3(sgrid(n)), dim3(256), 0, s, g.V + n, n,
                           1.0 / (std::sqrt(2.0) * n2));
        PPA_HIP(hipGetLastError());
    } else {
        set_unit(n, b, g.V, g.dpart, g.cw.nb, g.dout, s);
    }
    // (A - sigma I) v: the shift is the coefficient of the gathered vector
    // itself in the fused epilogue
    const bool sh = sigma != 0.0;
    auto op = [&](const double* vj, double* y) {
        if (b2) {
            launch_fused_spmv(A, VecT::F64, VecT::F64, -sigma, sh ? vj : nullptr, 1.0, vj, 0.0,
                              nullptr, 0.0, nullptr, y, s);
            launch_fused_spmv(A, VecT::F64, VecT::F64, -sigma, sh ? vj + n : nullptr, 1.0, vj + n,
                              0.0, nullptr, 0.0, nullptr, y + n, s);
        } else if (roots1.empty()) {
            launch_fused_spmv(A, VecT::F64, VecT::F64, -sigma, sh ? vj : nullptr, 1.0, vj, 0.0,
                              nullptr, 0.0, nullptr, y, s);
        } else {
            apply_tau(A, roots1, vj, y, g.aw, s, sigma);
        }
    };
    int64_t dots = 0, vops = 0;
    arnoldi_steps(N, 0, d, lowsync, g.V, g.ld, g.w, g.H, d + 1, g.ub0, g.ub1, g.cw, s, op,
                  [](int, int) {}, dots, vops);
    std::vector<double> H((size_t)(d + 1) * d);
    PPA_HIP(hipMemcpyAsync(H.data(), g.H, H.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    PPA_HIP(hipStreamSynchronize(s));
    for (double e : H)
        if (!std::isfinite(e)) fail(PPA_ERR_NONFINITE, "GMRES: non-finite Hessenberg entry");
    int deff = d;
    for (int j = 0; j < d; ++j) {
        double colsq = 0.0;
        for (int i = 0; i <= j + 1; ++i) colsq += H[i + (size_t)j * (d + 1)] * H[i + (size_t)j * (d + 1)];
        if (H[j + 1 + (size_t)j * (d + 1)] <= kBreakdownTol * std::sqrt(colsq)) {
            deff = j + 1;
            break;
        }
    }
    Hbar.assign((size_t)(deff + 1) * deff, 0.0);
    for (int j = 0; j < deff; ++j)
        for (int i = 0; i <= std::min(j + 1, deff); ++i) {
            if (i == deff && deff < d) continue;   // breakdown: zero last row
            Hbar[i + (size_t)j * (deff + 1)] = H[i + (size_t)j * (d + 1)];
        }
    return deff;
}

}  // namespace

// ---------------------------------------------------------------- build API
size_t poly_build_ws(int64_t n, int d, bool dbl) {
    Carver c(nullptr, 0);
    GmresWs g;
    carve_gmres(c, n, d, dbl, g);
    return c.bytes();
}

int poly_build(const Matrix& A, int d1, int d2, const double* b, void* ws, size_t ws_bytes,
               hipStream_t s, Poly& out, double sigma, bool lowsync) {
    const bool dbl = d2 > 0;
    const int dmax = std::max(d1, d2);
    PPA_REQUIRE(d1 >= 1 && dmax <= CGS_JMAX_ALL - 2, "polynomial degree out of range");
    Carver c(ws, ws_bytes);
    GmresWs g;
    carve_gmres(c, A.n, dmax, dbl, g);
    c.check();
    int status = PPA_OK;
    std::vector<double> Hb;
    out.shift = sigma;
    int de = gmres_cycle(A, {}, d1, b, nullptr, sigma, g, s, Hb, lowsync);
    if (de < d1) status = PPA_WARN_DEGREE_REDUCED;
    std::vector<cplx> r1 = leja_order(harmonic_ritz(de, Hb));
    if (!dbl) {
        out.roots = r1;
        out.roots1.clear();
        return status;
    }
    de = gmres_cycle(A, r1, d2, b, nullptr, sigma, g, s, Hb, lowsync);
    if (de < d2) status = PPA_WARN_DEGREE_REDUCED;
    out.roots1 = r1;
    out.roots = leja_order(harmonic_ritz(de, Hb));
    return status;
}

// ---------------------------------------------------------------- Arnoldi
namespace {

struct EigsWs {
    double* V = nullptr;
    double* V2 = nullptr;
    int64_t ld = 0;
    double* w = nullptr;
    ApplyWs aw64, aw32;
    Cgs2Ws cw;
    double* Hd = nullptr;
    double* Qd = nullptr;
    double* Y = nullptr;
    double* AY = nullptr;
    double* dpart = nullptr;
    double* dout = nullptr;
    int* cmap = nullptr;
    double* cscale = nullptr;
    int ycols = 0;
};

void carve_eigs(Carver& c, const Matrix& A, const Poly* p, const ppa_eigs_opts& o, EigsWs& e) {
    const int64_t n = A.n;
    e.ld = col_ld(n);
    e.V = c.take<double>((size_t)e.ld * (o.m + 1));
    e.V2 = c.take<double>((size_t)e.ld * (o.m + 1));
    e.w = c.take<double>((size_t)n);
    if (p) {
        carve_apply(c, n, *p, VecT::F64, e.aw64);
        if (o.precision == PPA_MIXED) carve_apply(c, n, *p, VecT::F32, e.aw32);
    }
    carve_cgs2(c, n, e.cw);
    e.Hd = c.take<double>((size_t)(o.m + 1) * o.m);
    // restart Q' ((m+1) x (k+1)) and Ritz coefficients G (m x 2 nev) share it
    e.Qd = c.take<double>((size_t)(o.m + 1) * std::max(o.m + 1, 2 * o.nev));
    e.ycols = 2 * o.nev;
    e.Y = c.take<double>((size_t)e.ld * e.ycols);
    e.AY = c.take<double>((size_t)e.ld * e.ycols);
    e.dpart = c.take<double>((size_t)MAX_DOTS * ritz_blocks(n));
    e.dout = c.take<double>(MAX_DOTS);
    e.cmap = c.take<int>((size_t)2 * o.nev);
    e.cscale = c.take<double>((size_t)2 * o.nev);
}

}  // namespace

size_t eigs_ws(const Matrix& A, const Poly* p, const ppa_eigs_opts& o) {
    Carver c(nullptr, 0);
    EigsWs e;
    carve_eigs(c, A, p, o, e);
    return c.bytes();
}

int eigs(const Matrix& A, const Poly* p, const ppa_eigs_opts& o, const double* v0, void* ws,
         size_t ws_bytes, hipStream_t s, ppa_eigs_result& r) {
    const int m = o.m, k = o.k, nev = o.nev;
    PPA_REQUIRE(m >= 2 && m <= 64, "eigs: m must be in [2, 64]");
    PPA_REQUIRE(nev >= 1 && nev <= k && k < m, "eigs: need 1 <= nev <= k < m");
    PPA_REQUIRE(nev <= 32, "eigs: nev must be <= 32");
    PPA_REQUIRE(o.max_cycles >= 1, "eigs: max_cycles must be >= 1");
    PPA_REQUIRE(o.precision == PPA_F64 || o.precision == PPA_MIXED, "eigs: precision must be F64 or MIXED");
    PPA_REQUIRE(o.precision == PPA_F64 || (p && A.v32), "eigs: MIXED needs a polynomial and FP32 values");
    PPA_REQUIRE(r.lam_re && r.lam_im && r.resid, "eigs: result arrays are required");
    const int64_t n = A.n;
    PPA_REQUIRE(n >= m + 1, "eigs: n must exceed m");
    Carver c(ws, ws_bytes);
    EigsWs e;
    carve_eigs(c, A, p, o, e);
    c.check();
    const double anorm = o.anorm > 0.0 ? o.anorm : A.norm_inf;
    const double rtol_abs = o.rtol * anorm;
    const double target = p ? 1.0 : 0.0;
    const int nb = e.cw.nb;

    // operator counts per application (same convention as the oracle)
    int64_t op_mvps = 1, op_vops = 0;
    if (p) {
        if (p->is_double()) {
            op_mvps = (int64_t)p->roots1.size() * p->roots.size();
            op_vops = (int64_t)p->roots.size() * ((int64_t)p->roots1.size() + 2);
        } else {
            op_mvps = p->roots.size();
            op_vops = p->roots.size();
        }
    }
    int64_t mvps = 0, dots = 0, vops = 0, passes = 0, passes32 = 0;
    double spmv_bytes = 0.0;
    bool fp32 = o.precision == PPA_MIXED;
    const bool timing = (o.flags & PPA_FLAG_TIMING) != 0;
    const bool harmonic = (o.flags & PPA_FLAG_HARMONIC) != 0;
    const bool lowsync = (o.flags & PPA_FLAG_LOWSYNC) != 0;
    struct Events {
        std::vector<hipEvent_t> ev;
        ~Events() {
            for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        }
    } tev;
    if (timing) {
        tev.ev.resize(3 * (size_t)(m + 1));
        for (auto& x : tev.ev) PPA_HIP(hipEventCreate(&x));
    }
    double t_apply = 0.0, t_cgs = 0.0;
    int fp32_cycles = 0;

    // stream of the Krylov steps: s, or the capture stream while a cycle's
    // steps are recorded into a graph
    hipStream_t cur = s;
    auto apply_op = [&](const double* x, double* y) {
        if (!p) {
            spmv_bytes += launch_fused_spmv(A, VecT::F64, VecT::F64, 0.0, nullptr, 1.0, x, 0.0, nullptr,
                                            0.0, nullptr, y, cur);
        } else if (fp32) {
            spmv_bytes += apply_poly(A, *p, VecT::F64, x, VecT::F64, y, VecT::F32, e.aw32, cur);
        } else {
            spmv_bytes += apply_poly(A, *p, VecT::F64, x, VecT::F64, y, VecT::F64, e.aw64, cur);
        }
        mvps += op_mvps;
        vops += op_vops;
        passes += op_mvps;
        if (fp32 && p) passes32 += op_mvps;
    };
    // HIP graphs of a cycle's Krylov steps, keyed by the start column, the
    // basis buffer (the restart swaps two) and the operator's precision; a
    // replay adds the counters the recorded launches added
    const bool graph = (o.flags & PPA_FLAG_GRAPH) != 0 && !timing;
    struct CycleGraph {
        int j0;
        const double* V;
        bool fp32;
        hipGraphExec_t exec;
        int64_t dm, dd, dv, dp, dp32;
        double db;
    };
    struct Graphs {
        std::vector<CycleGraph> g;
        hipStream_t cs = nullptr;
        ~Graphs() {
            for (auto& x : g) (void)hipGraphExecDestroy(x.exec);
            if (cs) (void)hipStreamDestroy(cs);
        }
    } graphs;
    bool graph_ok = graph;
    constexpr size_t kMaxGraphs = 4;

    launch_zero(e.Hd, (int64_t)(m + 1) * m, s);
    set_unit(n, v0, e.V, e.dpart, nb, e.dout, s);
    int j0 = 0;
    std::vector<double> H((size_t)(m + 1) * m);
    std::vector<double> hist;
    struct RitzOut {
        std::vector<cplx> mu;
        std::vector<double> res;
        std::vector<double> ynorm;
    };
    RitzOut last;
    RitzPlan lastw;
    std::vector<cplx> lastnu;
    // Ritz test of the pairs planned in R (Y = V_vcols Gw): Y and A Y on the
    // device, Rayleigh quotients mu = y* A y and residual norms ||A y - mu y||
    // for unit y
    auto ritz_test = [&](const RitzPlan& R, int vcols) {
        PPA_HIP(hipMemcpyAsync(e.Qd, R.Gw.data(), R.Gw.size() * sizeof(double), hipMemcpyHostToDevice, s));
        launch_gemm_tall(n, vcols, R.ycols, e.V, e.ld, e.Qd, e.Y, e.ld, s);
        launch_spmm_cols(A, e.Y, e.ld, R.ycols, e.AY, s);
        const std::vector<DotSpec> dspec = ritz_dots(R);
        std::vector<double> dv(dspec.size());
        for (size_t off = 0; off < dspec.size(); off += MAX_DOTS) {
            DotList L{};
            L.count = (int)std::min<size_t>(MAX_DOTS, dspec.size() - off);
            for (int t = 0; t < L.count; ++t) {
                const DotSpec& q = dspec[off + t];
                L.a[t] = e.Y + (size_t)q.a * e.ld;
                L.b[t] = (q.kind == 1 ? e.Y : e.AY) + (size_t)q.b * e.ld;
            }
            launch_dots(n, L, e.dpart, ritz_blocks(n), e.dout, s);
            PPA_HIP(hipMemcpyAsync(dv.data() + off, e.dout, L.count * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        PPA_HIP(hipStreamSynchronize(s));
        RitzOut Rr;
        ritz_mu(R, dv, Rr.mu, Rr.ynorm);
        mvps += ritz_mvps(R);
        // residual norms ||A y - mu y|| / ||y||
        {
            const std::vector<ComboSpec> cs = ritz_combos(R, Rr.mu);
            const int nl = (int)cs.size();
            std::vector<double> rn(nl);
            for (int done = 0; done < nl;) {
                ComboList P{};
                P.count = std::min(MAX_COMBOS, nl - done);
                for (int q = 0; q < P.count; ++q)
                    for (int t = 0; t < 3; ++t) {
                        const ComboSpec& c = cs[done + q];
                        P.v[q][t] = t < c.nterms ? (c.kind[t] == 0 ? e.AY : e.Y) + (size_t)c.col[t] * e.ld : nullptr;
                        P.c[q][t] = t < c.nterms ? c.c[t] : 0.0;
                    }
                launch_combo_norms(n, P, e.dpart, ritz_blocks(n), e.dout, s);
                PPA_HIP(hipMemcpyAsync(rn.data() + done, e.dout, P.count * sizeof(double), hipMemcpyDeviceToHost, s));
                done += P.count;
            }
            PPA_HIP(hipStreamSynchronize(s));
            ritz_resid(R, cs, rn, Rr.ynorm, Rr.res);
        }
        return Rr;
    };
    bool converged = false, broke = false;
    int cycle = 0;
    for (cycle = 1; cycle <= o.max_cycles; ++cycle) {
        if (fp32) ++fp32_cycles;
        // the delayed form keeps its candidates in two columns of V2, which is
        // free until the restart
        auto steps = [&](hipStream_t st) {
            cur = st;
            arnoldi_steps(n, j0, m, lowsync, e.V, e.ld, e.w, e.Hd, m + 1, e.V2, e.V2 + e.ld, e.cw, st,
                          apply_op,
                          [&](int j, int phase) {
                              if (timing) PPA_HIP(hipEventRecord(tev.ev[3 * j + phase], st));
                          },
                          dots, vops);
            cur = s;
        };
        const CycleGraph* hit = nullptr;
        if (graph_ok)
            for (const auto& x : graphs.g)
                if (x.j0 == j0 && x.V == e.V && x.fp32 == fp32) hit = &x;
        if (hit) {
            PPA_HIP(hipGraphLaunch(hit->exec, s));
            mvps += hit->dm;
            dots += hit->dd;
            vops += hit->dv;
            passes += hit->dp;
            passes32 += hit->dp32;
            spmv_bytes += hit->db;
        } else if (graph_ok && graphs.g.size() < kMaxGraphs) {
            if (!graphs.cs) PPA_HIP(hipStreamCreateWithFlags(&graphs.cs, hipStreamNonBlocking));
            const int64_t m0 = mvps, d0 = dots, v0c = vops, p0 = passes, q0 = passes32;
            const double b0 = spmv_bytes;
            PPA_HIP(hipStreamBeginCapture(graphs.cs, hipStreamCaptureModeThreadLocal));
            hipGraph_t gr = nullptr;
            try {
                steps(graphs.cs);
            } catch (...) {
                cur = s;
                (void)hipStreamEndCapture(graphs.cs, &gr);
                if (gr) (void)hipGraphDestroy(gr);
                (void)hipGetLastError();
                throw;
            }
            PPA_HIP(hipStreamEndCapture(graphs.cs, &gr));
            hipGraphExec_t ex = nullptr;
            const hipError_t ie = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            PPA_HIP(ie);
            graphs.g.push_back({j0, e.V, fp32, ex, mvps - m0, dots - d0, vops - v0c, passes - p0,
                                passes32 - q0, spmv_bytes - b0});
            PPA_HIP(hipGraphLaunch(ex, s));
        } else {
            steps(s);
        }
        PPA_HIP(hipMemcpyAsync(H.data(), e.Hd, H.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        PPA_HIP(hipStreamSynchronize(s));
        if (timing) {
            for (int j = j0; j < m; ++j) {
                float a = 0.f, b = 0.f;
                PPA_HIP(hipEventElapsedTime(&a, tev.ev[3 * j], tev.ev[3 * j + 1]));
                PPA_HIP(hipEventElapsedTime(&b, tev.ev[3 * j + 1], tev.ev[3 * j + 2]));
                t_apply += a;
                t_cgs += b;
            }
        }
        for (double x : H)
            if (!std::isfinite(x)) fail(PPA_ERR_NONFINITE, "Arnoldi: non-finite Hessenberg entry");
        int mc = m;
        for (int j = j0; j < m; ++j) {
            double colsq = 0.0;
            for (int i = 0; i <= j + 1; ++i) colsq += H[i + (size_t)j * (m + 1)] * H[i + (size_t)j * (m + 1)];
            if (H[j + 1 + (size_t)j * (m + 1)] <= kBreakdownTol * std::sqrt(colsq)) {
                mc = j + 1;
                broke = true;
                break;
            }
        }
        // Ritz pairs of the operator
        std::vector<double> Hm((size_t)mc * mc);
        for (int jj = 0; jj < mc; ++jj)
            for (int i = 0; i < mc; ++i) Hm[i + (size_t)jj * mc] = H[i + (size_t)jj * (m + 1)];
        RitzPlan R = plan_ritz(Hm, mc, nev, target, harmonic && mc == m,
                               mc == m ? H[m + (size_t)(m - 1) * (m + 1)] : 0.0);
        const int nw = R.nw;
        RitzOut Rr = ritz_test(R, mc);
        double mx = 0.0;
        for (int i = 0; i < nw; ++i) mx = std::max(mx, Rr.res[i]);
        hist.push_back(mx);
        last = Rr;
        lastw = R;
        lastnu.assign(R.nu.begin(), R.nu.begin() + nw);
        converged = (nw == nev) && mx <= rtol_abs;
        if (converged || broke || cycle == o.max_cycles) break;

        if (fp32) {
            // leave the FP32 phase when the wanted residuals reach the FP32
            // floor, or stop improving within three decades of it (slow
            // progress far above the floor is the method's, not the
            // precision's, and FP64 cycles would not speed it up)
            if (leave_fp32(hist, anorm)) {
                fp32 = false;
                // closing FP64 Rayleigh-Ritz with A itself on the FP32-built
                // basis V_{m+1} (FP64 storage, orthonormal to FP64 rounding):
                // K = V^T A V, its Ritz pairs nearest the target, tested on A
                // as every cycle's pairs are.  When they all meet rtol the
                // solve ends here; otherwise the FP64 cycles start from v0.
                // Costs m + 1 products with A and (m + 1)^2 inner products,
                // against m factors of pi per cycle.
                const int J = mc + 1;
                launch_spmm_cols(A, e.V, e.ld, J, e.V2, s);
                launch_gram(n, J, e.V, e.ld, e.V2, J, e.Qd, e.cw, s);
                std::vector<double> K((size_t)J * J);
                PPA_HIP(hipMemcpyAsync(K.data(), e.Qd, K.size() * sizeof(double), hipMemcpyDeviceToHost, s));
                PPA_HIP(hipStreamSynchronize(s));
                for (double x : K)
                    if (!std::isfinite(x)) fail(PPA_ERR_NONFINITE, "closing Rayleigh-Ritz: non-finite projection");
                mvps += J;
                dots += (int64_t)J * J;
                const RitzPlan R2 = plan_ritz(K, J, nev, p ? p->shift : 0.0);
                const RitzOut Rr2 = ritz_test(R2, J);
                double mx2 = 0.0;
                for (int i = 0; i < R2.nw; ++i) mx2 = std::max(mx2, Rr2.res[i]);
                hist.back() = std::min(mx, mx2);
                if (R2.nw == nev && mx2 <= rtol_abs) {
                    last = Rr2;
                    lastw = R2;
                    lastnu.assign(R2.nu.begin(), R2.nu.begin() + R2.nw);
                    converged = true;
                    break;
                }
                // otherwise the FP64 cycles start again from v0: a restart
                // from these Ritz vectors carries the copies of multiple
                // eigenvalues that the FP32 rounding brought in, and when the
                // wanted set ends inside such a cluster the FP64 cycles keep
                // trading its members in and out instead of converging
                launch_zero(e.Hd, (int64_t)(m + 1) * m, s);
                set_unit(n, v0, e.V, e.dpart, nb, e.dout, s);
                j0 = 0;
                continue;
            }
        }

        // thick restart: keep k (k-1 if a conjugate pair would be split)
        const RestartPlan RP = plan_restart(R, Hm, H[m + (size_t)(m - 1) * (m + 1)], m, k);
        PPA_HIP(hipMemcpyAsync(e.Qd, RP.Qp.data(), RP.Qp.size() * sizeof(double), hipMemcpyHostToDevice, s));
        launch_gemm_tall(n, m + 1, RP.kk + 1, e.V, e.ld, e.Qd, e.V2, e.ld, s);
        std::swap(e.V, e.V2);
        PPA_HIP(hipMemcpyAsync(e.Hd, RP.Hn.data(), RP.Hn.size() * sizeof(double), hipMemcpyHostToDevice, s));
        j0 = RP.kk;
    }
    if (cycle > o.max_cycles) cycle = o.max_cycles;

    // outputs sorted by |mu| (ties: Re, then Im)
    const int nw = (int)last.mu.size();
    std::vector<int> ord(nw);
    std::iota(ord.begin(), ord.end(), 0);
    // returned by distance to the target (the polynomial's shift; 0: the origin)
    const double tgt = p ? p->shift : 0.0;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
        const double ma = std::abs(last.mu[a] - tgt), mb = std::abs(last.mu[b] - tgt);
        if (ma != mb) return ma < mb;
        if (last.mu[a].real() != last.mu[b].real()) return last.mu[a].real() < last.mu[b].real();
        return last.mu[a].imag() < last.mu[b].imag();
    });
    int nconv = 0;
    double maxres = 0.0;
    for (int t = 0; t < nev; ++t) {
        if (t < nw) {
            const int i = ord[t];
            r.lam_re[t] = last.mu[i].real();
            r.lam_im[t] = last.mu[i].imag();
            r.resid[t] = last.res[i];
            if (r.ritz_re) r.ritz_re[t] = lastnu[i].real();
            if (r.ritz_im) r.ritz_im[t] = lastnu[i].imag();
            if (last.res[i] <= rtol_abs) ++nconv;
            maxres = std::max(maxres, last.res[i]);
        } else {
            r.lam_re[t] = r.lam_im[t] = std::nan("");
            r.resid[t] = std::nan("");
        }
    }
    if (r.X_d && nw > 0) {
        std::vector<int> cre(nw), cim(nw);
        std::vector<double> sc(2 * nw);
        for (int t = 0; t < nw; ++t) {
            const int i = ord[t];
            cre[t] = lastw.cre[i];
            cim[t] = lastw.cim[i];
            const double inv = 1.0 / last.ynorm[i];
            sc[2 * t] = inv;
            sc[2 * t + 1] = (lastw.dup[i] ? -1.0 : 1.0) * inv;
        }
        // Y still holds the wanted columns of the last cycle
        std::vector<int> maps(2 * nw);
        for (int t = 0; t < nw; ++t) {
            maps[t] = cre[t];
            maps[nw + t] = cim[t];
        }
        PPA_HIP(hipMemcpyAsync(e.cmap, maps.data(), maps.size() * sizeof(int), hipMemcpyHostToDevice, s));
        PPA_HIP(hipMemcpyAsync(e.cscale, sc.data(), sc.size() * sizeof(double), hipMemcpyHostToDevice, s));
        launch_copy_cols_complex(n, e.Y, e.ld, e.cmap, e.cmap + nw, e.cscale, nw, r.X_d, s);
        PPA_HIP(hipStreamSynchronize(s));
    }
    r.nconv = nconv;
    r.cycles = cycle;
    r.mvps = mvps;
    r.dots = dots;
    r.vops = vops;
    r.max_resid = maxres;
    r.fp32_cycles = fp32_cycles;
    r.spmv_passes = passes;
    r.spmv_passes_f32 = passes32;
    r.spmv_bytes = spmv_bytes;
    r.t_apply_ms = t_apply;
    r.t_cgs_ms = t_cgs;
    if (converged) return PPA_OK;
    if (broke) return PPA_WARN_BREAKDOWN;
    return PPA_WARN_NOT_CONVERGED;
}

// ---------------------------------------------------------------- safeguards
// Sections 5-6: a GMRES polynomial from a damped start vector A^p b (+ alpha
// b), optionally from two start vectors, optionally checked by the
// Ideal-Order-Condition heuristic: one Arnoldi(m,k) cycle on pi(A) from b,
// Ritz values ordered by |1 - nu|, Rayleigh quotients mu_j = y_j^* A y_j for
// j <= k, and the test |mu_1| <= ... <= |mu_nev| < min_{nev < j <= k} |mu_j|.
// On failure the start vector is damped once more (A b in place of b), and
// while the test still fails the degree is halved (keeping the damped start
// vector), down to d = 1.
namespace {

struct BuildExWs {
    double* s1 = nullptr;
    double* s2 = nullptr;
    double* tmp = nullptr;
    GmresWs g;
    void* ews = nullptr;
    size_t ews_bytes = 0;
};

ppa_eigs_opts test_opts(const ppa_poly_build_opts& o) {
    ppa_eigs_opts t{};
    t.m = o.test_m;
    t.k = o.test_k;
    t.nev = o.test_k;
    t.max_cycles = 1;
    t.rtol = 0.0;
    t.anorm = 0.0;
    t.precision = PPA_F64;
    t.flags = o.flags & PPA_FLAG_LOWSYNC;
    return t;
}

void carve_build_ex(Carver& c, const Matrix& A, const ppa_poly_build_opts& o, bool two,
                    BuildExWs& w) {
    const int64_t n = A.n;
    w.s1 = c.take<double>((size_t)n);
    if (two) w.s2 = c.take<double>((size_t)n);
    w.tmp = c.take<double>((size_t)n);
    carve_gmres(c, two ? 2 * n : n, o.d, false, w.g);
    if (o.test_m > 0) {
        Poly single;
        single.roots.assign(1, cplx(1.0, 0.0));
        w.ews_bytes = eigs_ws(A, &single, test_opts(o));
        w.ews = c.take<char>(w.ews_bytes);
    }
}

// dst = A^power b (+ alpha b on the last pass), power 0..2
void damp_start(const Matrix& A, const double* b, int power, double alpha, double* dst, double* tmp,
                hipStream_t s) {
    if (power == 0) {
        hipLaunchKernelGGL(k_copy, dim3(sgrid(A.n)), dim3(256), 0, s, b, dst, A.n);
        PPA_HIP(hipGetLastError());
        return;
    }
    const double* cur = b;
    for (int p = 0; p < power; ++p) {
        const bool last = p == power - 1;
        double* out = last ? dst : tmp;
        launch_fused_spmv(A, VecT::F64, VecT::F64, last ? alpha : 0.0,
                          (last && alpha != 0.0) ? b : nullptr, 1.0, cur, 0.0, nullptr, 0.0,
                          nullptr, out, s);
        cur = out;
    }
}

}  // namespace

size_t poly_build_ex_ws(const Matrix& A, const ppa_poly_build_opts& o, bool two) {
    Carver c(nullptr, 0);
    BuildExWs w;
    carve_build_ex(c, A, o, two, w);
    return c.bytes();
}

int poly_build_ex(const Matrix& A, const ppa_poly_build_opts& o, const double* b, const double* b2,
                  void* ws, size_t ws_bytes, hipStream_t s, Poly& out, ppa_poly_build_info& info) {
    PPA_REQUIRE(o.d >= 1 && o.d <= CGS_JMAX_ALL - 2, "polynomial degree out of range");
    PPA_REQUIRE(o.damp >= 0 && o.damp <= 2, "damping power must be 0, 1 or 2");
    const bool test = o.test_m > 0;
    if (test) {
        PPA_REQUIRE(o.test_m >= 2 && o.test_m <= 64 && o.test_nev >= 1 && o.test_nev <= o.test_k &&
                        o.test_k < o.test_m && o.test_k <= 32,
                    "order test: need 1 <= nev <= k < m <= 64, k <= 32");
        PPA_REQUIRE(A.n >= o.test_m + 1, "order test: n must exceed m");
    }
    Carver c(ws, ws_bytes);
    BuildExWs w;
    carve_build_ex(c, A, o, b2 != nullptr, w);
    c.check();
    int d = o.d, power = o.damp, attempts = 0, status = PPA_OK;
    int held = -1;
    for (;;) {
        damp_start(A, b, power, o.alpha, w.s1, w.tmp, s);
        if (b2) damp_start(A, b2, power, o.alpha, w.s2, w.tmp, s);
        std::vector<double> Hb;
        const int de = gmres_cycle(A, {}, d, w.s1, b2 ? w.s2 : nullptr, o.shift, w.g, s, Hb,
                                   (o.flags & PPA_FLAG_LOWSYNC) != 0);
        status = de < d ? PPA_WARN_DEGREE_REDUCED : PPA_OK;
        Poly p;
        p.roots = leja_order(harmonic_ritz(de, Hb));
        p.shift = o.shift;
        ++attempts;
        if (test) {
            const ppa_eigs_opts t = test_opts(o);
            std::vector<double> lre(t.nev), lim(t.nev), res(t.nev), nre(t.nev), nim(t.nev);
            ppa_eigs_result r{};
            r.lam_re = lre.data();
            r.lam_im = lim.data();
            r.resid = res.data();
            r.ritz_re = nre.data();
            r.ritz_im = nim.data();
            (void)eigs(A, &p, t, b, w.ews, w.ews_bytes, s, r);
            // the returned pairs back in the order of |1 - nu|
            std::vector<cplx> nu, mu;
            for (int i = 0; i < t.nev; ++i)
                if (std::isfinite(lre[i])) {
                    nu.emplace_back(nre[i], nim[i]);
                    mu.emplace_back(lre[i], lim[i]);
                }
            const std::vector<int> ord = sort_ritz(nu, 1.0);
            const int kk = (int)ord.size(), nev = std::min(o.test_nev, kk);
            bool ok = nev >= 1;
            // distances to the target mu = shift (0: the origin)
            auto dist = [&](int i) { return std::abs(mu[ord[i]] - o.shift); };
            for (int i = 0; ok && i + 1 < nev; ++i) ok = dist(i) <= dist(i + 1);
            for (int i = nev; ok && i < kk; ++i) ok = dist(nev - 1) < dist(i);
            held = ok ? 1 : 0;
        }
        if (!test || held == 1 || d == 1) {
            out.roots = std::move(p.roots);
            out.roots1.clear();
            out.shift = p.shift;
            break;
        }
        if (power == o.damp && power < 2)
            ++power;          // damp: A b in place of b
        else
            d = std::max(1, d / 2);
    }
    info.degree = (int)out.roots.size();
    info.damp = power;
    info.attempts = attempts;
    info.held = held;
    return status;
}

}  // namespace ppa
