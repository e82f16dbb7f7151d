// Batched engine for many small solves (the served form): one launch runs a
// phase of every admitted solve, one workgroup per solve.
//
// A small solve (n up to a few 10^4) cannot fill the chip and its kernels
// would be launch-bound, so the engine packs them: workgroup b reads slot
// descriptor b and runs, inside the workgroup, that solve's next phase:
//   BUILD  GMRES(d) steps on A (section 2, step 1(a)),
//   CYCLE  Krylov steps on pi(A): d fused passes plus CGS2 per step, up to a
//          pass budget, optionally after the thick-restart product V Q,
//   TEST   Ritz vectors Y = V_m G, A Y, Rayleigh quotients and residual norms
//          (section 4),
//   RR     the closing FP64 Rayleigh-Ritz projection of a mixed-precision
//          solve, K = V^T A V over the basis its FP32 cycles built,
// and the host handles the small projected problems between launches (roots,
// Ritz pairs, restart), sharing that logic with the single-solve driver.
// Solves join free slots and leave finished ones between launches
// (continuous batching).  Every reduction runs inside one workgroup in a fixed
// order, so a solve's result does not depend on what else is in the batch.
// The per-row sums of a pass follow the same order and expression as the
// main SpMV kernel.  A mixed-precision solve applies pi(A) in FP32 (values,
// vectors and sums; the last factor's result stored to the FP64 basis), as
// the single-solve path does, and everything else in FP64.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "ppa_internal.hpp"

namespace ppa {

namespace {

#ifndef PPA_BATCH_WG
#define PPA_BATCH_WG 1024
#endif
constexpr int BWG = PPA_BATCH_WG; // threads per workgroup
constexpr int BNW = BWG / 64;
constexpr int BMAXJ = 128;        // largest basis (GMRES degree or m) + 1
constexpr int BMAXW = 32;         // largest nev
constexpr double kBTol = 1e-14;   // breakdown threshold, as in the main path

enum : int { PH_IDLE = 0, PH_BUILD = 1, PH_CYCLE = 2, PH_TEST = 3, PH_RR = 4 };

}  // namespace

struct BSlot {
    const int32_t* rowptr;
    const int32_t* colind;
    const double* val;
    double* V;        // current basis, column-major, leading dimension ld
    double* V2;       // restart target
    double* w;        // operator output
    double* t1;       // temporaries (polynomial chain, CGS2)
    double* t2;
    double* t3;
    double* H;        // projected matrix, ldh rows
    double* Y;        // Ritz vectors (ycols columns)
    double* AY;
    double* Q;        // coefficient matrix qin x qout (restart or Ritz)
    double* out;      // TEST results: mu_re, mu_im, res, ynorm (BMAXW each)
    const double* start;
    const double* rre;   // polynomial roots, application order
    const double* rim;
    const float* val32;  // FP32 copy of the values (mixed precision), else null
    float* f1;           // FP32 chain vectors (mixed precision)
    float* f2;
    float* f3;
    float* f4;
    int n, ld, ldh;
    int phase, init, restart, use_poly;
    int f32;             // CYCLE: pi(A) in FP32
    int j, jend, budget, deg;
    int qin, qout;
    int nw, ycols;
    int wcre[BMAXW], wcim[BMAXW], wdup[BMAXW];
    int j_done;
    int pad;
};

namespace {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block sum of up to 8 values per thread; every thread receives the totals.
// red must hold 8 * BNW doubles; out (LDS) receives cnt totals.
__device__ void bsum8(const double (&acc)[8], int cnt, double* red, double* out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (c < cnt) {
            const double v = wsum(acc[c]);
            if (lane == 0) red[wv * 8 + c] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < cnt) {
        double t = 0.0;
        for (int q = 0; q < BNW; ++q) t += red[q * 8 + threadIdx.x];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

__device__ double bsum1(double v, double* red, double* tmp) {
    double a[8] = {v, 0, 0, 0, 0, 0, 0, 0};
    bsum8(a, 1, red, tmp);
    return tmp[0];
}

// out = alpha x + beta (A u) + gamma z over all rows; per-row sum in column
// order, epilogue written as in the main kernel.
__device__ void wg_pass(const BSlot& S, double alpha, const double* x, double beta,
                        const double* u, double gamma, const double* z, double* out) {
    for (int r = threadIdx.x; r < S.n; r += BWG) {
        const int a = S.rowptr[r], e = S.rowptr[r + 1];
        double s = 0.0;
        for (int k = a; k < e; ++k) s += S.val[k] * u[S.colind[k]];
        const double xv = x ? x[r] : 0.0, zv = z ? z[r] : 0.0;
        out[r] = beta * s + alpha * xv + gamma * zv + 0.0 * 0.0;
    }
    __syncthreads();
}

// FP32 form of wg_pass for the mixed-precision chain (no z term: the chain
// never uses it); the result goes to out32, or, when out64 is given, is
// stored there widened to FP64.
__device__ void wg_pass32(const BSlot& S, float alpha, const float* x, float beta, const float* u,
                          float* out32, double* out64) {
    for (int r = threadIdx.x; r < S.n; r += BWG) {
        const int a = S.rowptr[r], e = S.rowptr[r + 1];
        float s = 0.0f;
        for (int k = a; k < e; ++k) s += S.val32[k] * u[S.colind[k]];
        const float xv = x ? x[r] : 0.0f;
        const float o = beta * s + alpha * xv + 0.0f * 0.0f;
        if (out64)
            out64[r] = (double)o;
        else
            out32[r] = o;
    }
    __syncthreads();
}

__device__ float* pick3f(const BSlot& S, const float* a, const float* b) {
    float* c[3] = {S.f1, S.f2, S.f3};
    for (int i = 0; i < 3; ++i)
        if (c[i] != a && c[i] != b) return c[i];
    return S.f3;
}

// y = pi(A) v with the chain in FP32: v rounded to FP32 once, every factor
// in FP32 (coefficients formed in FP64, then rounded), the last factor's
// result widened into y
__device__ void wg_apply32(const BSlot& S, const double* v, double* y) {
    for (int r = threadIdx.x; r < S.n; r += BWG) S.f4[r] = (float)v[r];
    __syncthreads();
    const float* cur = S.f4;
    int i = 0;
    while (i < S.deg) {
        const double re = S.rre[i], im = S.rim[i];
        const bool pair = im != 0.0;
        const bool last = i + (pair ? 2 : 1) >= S.deg;
        if (!pair) {
            float* nx = last ? nullptr : pick3f(S, cur, nullptr);
            wg_pass32(S, 1.0f, cur, (float)(-1.0 / re), cur, nx, last ? y : nullptr);
            cur = nx;
            i += 1;
        } else {
            const double q = re * re + im * im;
            float* sb = pick3f(S, cur, nullptr);
            wg_pass32(S, (float)(2.0 * re), cur, -1.0f, cur, sb, nullptr);
            float* nx = last ? nullptr : pick3f(S, cur, sb);
            wg_pass32(S, 1.0f, cur, (float)(-1.0 / q), sb, nx, last ? y : nullptr);
            cur = nx;
            i += 2;
        }
    }
}

__device__ double* pick3(const BSlot& S, const double* a, const double* b) {
    double* c[3] = {S.t1, S.t2, S.t3};
    for (int i = 0; i < 3; ++i)
        if (c[i] != a && c[i] != b) return c[i];
    return S.t3;
}

// y = pi(A) v, factors in order (real root: one pass; pair: two passes)
__device__ void wg_apply(const BSlot& S, const double* v, double* y) {
    const double* cur = v;
    int i = 0;
    while (i < S.deg) {
        const double re = S.rre[i], im = S.rim[i];
        const bool pair = im != 0.0;
        const bool last = i + (pair ? 2 : 1) >= S.deg;
        if (!pair) {
            double* nx = last ? y : pick3(S, cur, nullptr);
            wg_pass(S, 1.0, cur, -1.0 / re, cur, 0.0, nullptr, nx);
            cur = nx;
            i += 1;
        } else {
            const double q = re * re + im * im;
            double* sb = pick3(S, cur, nullptr);
            wg_pass(S, 2.0 * re, cur, -1.0, cur, 0.0, nullptr, sb);
            double* nx = last ? y : pick3(S, cur, sb);
            wg_pass(S, 1.0, cur, -1.0 / q, sb, 0.0, nullptr, nx);
            cur = nx;
            i += 2;
        }
    }
}

// h[0..j) = V^T w for the first j columns of V (block sums, 8 at a time)
__device__ void wg_proj(const BSlot& S, const double* V, int j, const double* w, double* h,
                        double* red) {
    for (int c0 = 0; c0 < j; c0 += 8) {
        const int cnt = min(8, j - c0);
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int r = threadIdx.x; r < S.n; r += BWG) {
            const double wr = w[r];
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c < cnt) acc[c] += V[(size_t)(c0 + c) * S.ld + r] * wr;
        }
        bsum8(acc, cnt, red, h + c0);
    }
}

// out = t - V h (first j columns); returns ||out||^2 (block sum)
__device__ double wg_update(const BSlot& S, const double* V, int j, const double* h, const double* t,
                            double* out, double* red, double* tmp) {
    double nrm = 0.0;
    for (int r = threadIdx.x; r < S.n; r += BWG) {
        double tv = t[r];
        for (int c = 0; c < j; ++c) tv -= V[(size_t)c * S.ld + r] * h[c];
        out[r] = tv;
        nrm += tv * tv;
    }
    __syncthreads();
    return bsum1(nrm, red, tmp);
}

// Orthogonalise w against V[:, 0:j] with one reorthogonalisation pass, write
// v_{j} = w_out / beta into V[:, j] and the Hessenberg column (j+1 entries).
__device__ void wg_cgs2(const BSlot& S, double* V, int j, const double* w, double* Hcol,
                        double* h1, double* h2, double* red, double* tmp) {
    wg_proj(S, V, j, w, h1, red);
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int r = threadIdx.x; r < S.n; r += BWG) a[0] += w[r] * w[r];
    bsum8(a, 1, red, tmp);
    const double w0 = sqrt(tmp[0]);
    wg_update(S, V, j, h1, w, S.t1, red, tmp);
    wg_proj(S, V, j, S.t1, h2, red);
    double* vn = V + (size_t)j * S.ld;
    const double b2 = wg_update(S, V, j, h2, S.t1, vn, red, tmp);
    const double beta = sqrt(b2);
    const double inv = (beta > kBTol * w0 && beta > 0.0) ? 1.0 / beta : 0.0;
    for (int r = threadIdx.x; r < S.n; r += BWG) vn[r] *= inv;
    if (threadIdx.x == 0) {
        for (int i = 0; i < j; ++i) Hcol[i] = h1[i] + h2[i];
        Hcol[j] = beta;
    }
    __syncthreads();
}

// dst[:, c] = V[:, 0:qin] Q[:, c] for c < qout (Q in LDS, qin x qout col-major)
__device__ void wg_gemm(const BSlot& S, const double* V, const double* Qs, int qin, int qout,
                        double* dst) {
    for (int r = threadIdx.x; r < S.n; r += BWG) {
        for (int c0 = 0; c0 < qout; c0 += 8) {
            double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int i = 0; i < qin; ++i) {
                const double v = V[(size_t)i * S.ld + r];
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if (c0 + c < qout) acc[c] += v * Qs[i + (c0 + c) * qin];
            }
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c0 + c < qout) dst[(size_t)(c0 + c) * S.ld + r] = acc[c];
        }
    }
    __syncthreads();
}

__device__ void wg_normalise(const BSlot& S, const double* src, double* dst, double* red, double* tmp) {
    double a = 0.0;
    for (int r = threadIdx.x; r < S.n; r += BWG) a += src[r] * src[r];
    const double nn = sqrt(bsum1(a, red, tmp));
    const double inv = nn > 0.0 ? 1.0 / nn : 0.0;
    for (int r = threadIdx.x; r < S.n; r += BWG) dst[r] = src[r] * inv;
    __syncthreads();
}

// dot of two columns, block sum
__device__ double wg_dot(const BSlot& S, const double* a, const double* b, double* red, double* tmp) {
    double s = 0.0;
    for (int r = threadIdx.x; r < S.n; r += BWG) s += a[r] * b[r];
    return bsum1(s, red, tmp);
}

// ||c0 v0 + c1 v1 + c2 v2||^2 (v2 may be null)
__device__ double wg_combo(const BSlot& S, const double* v0, double c0, const double* v1, double c1,
                           const double* v2, double c2, double* red, double* tmp) {
    double s = 0.0;
    for (int r = threadIdx.x; r < S.n; r += BWG) {
        double v = c0 * v0[r] + c1 * v1[r];
        if (v2) v += c2 * v2[r];
        s += v * v;
    }
    return bsum1(s, red, tmp);
}

__global__ __launch_bounds__(BWG) void k_batch(BSlot* __restrict__ slots) {
    __shared__ double red[8 * BNW];
    __shared__ double tmp[8];
    __shared__ double h1[BMAXJ], h2[BMAXJ];
    __shared__ double Qs[65 * 64];
    BSlot& S = slots[blockIdx.x];
    if (S.phase == PH_IDLE) return;
    if (S.phase == PH_RR) {
        // K = V^T (A V) over the first qin basis columns: A V into V2, then
        // column c of K (qin entries) into Q + c qin
        for (int c = 0; c < S.qin; ++c)
            wg_pass(S, 0.0, nullptr, 1.0, S.V + (size_t)c * S.ld, 0.0, nullptr, S.V2 + (size_t)c * S.ld);
        for (int c = 0; c < S.qin; ++c)
            wg_proj(S, S.V, S.qin, S.V2 + (size_t)c * S.ld, S.Q + (size_t)c * S.qin, red);
        if (threadIdx.x == 0) S.j_done = S.j;
        return;
    }
    if (S.phase == PH_BUILD || S.phase == PH_CYCLE) {
        double* V = S.V;
        if (S.restart) {
            // thick restart: V2 = V Q (Q staged in LDS), then continue on V2
            for (int i = threadIdx.x; i < S.qin * S.qout; i += BWG) Qs[i] = S.Q[i];
            __syncthreads();
            wg_gemm(S, S.V, Qs, S.qin, S.qout, S.V2);
            V = S.V2;
        }
        if (S.init) wg_normalise(S, S.start, V, red, tmp);
        int j = S.j, used = 0;
        const int cost = S.use_poly ? S.deg : 1;
        while (j < S.jend && (used == 0 || used + cost <= S.budget)) {
            const double* vj = V + (size_t)j * S.ld;
            if (S.use_poly && S.f32)
                wg_apply32(S, vj, S.w);
            else if (S.use_poly)
                wg_apply(S, vj, S.w);
            else
                wg_pass(S, 0.0, nullptr, 1.0, vj, 0.0, nullptr, S.w);
            wg_cgs2(S, V, j + 1, S.w, S.H + (size_t)j * S.ldh, h1, h2, red, tmp);
            used += cost;
            ++j;
        }
        if (threadIdx.x == 0) S.j_done = j;
        return;
    }
    // PH_TEST: Y = V G, A Y, Rayleigh quotients and residuals
    for (int i = threadIdx.x; i < S.qin * S.qout; i += BWG) Qs[i] = S.Q[i];
    __syncthreads();
    wg_gemm(S, S.V, Qs, S.qin, S.qout, S.Y);
    for (int c = 0; c < S.ycols; ++c)
        wg_pass(S, 0.0, nullptr, 1.0, S.Y + (size_t)c * S.ld, 0.0, nullptr, S.AY + (size_t)c * S.ld);
    double* mre = S.out;
    double* mim = S.out + BMAXW;
    double* res = S.out + 2 * BMAXW;
    double* yn = S.out + 3 * BMAXW;
    for (int i = 0; i < S.nw; ++i) {
        if (S.wdup[i]) {
            if (threadIdx.x == 0) {
                mre[i] = mre[i - 1];
                mim[i] = -mim[i - 1];
                res[i] = res[i - 1];
                yn[i] = yn[i - 1];
            }
            continue;
        }
        const double* Ya = S.Y + (size_t)S.wcre[i] * S.ld;
        const double* AYa = S.AY + (size_t)S.wcre[i] * S.ld;
        if (S.wcim[i] < 0) {
            const double yy = wg_dot(S, Ya, Ya, red, tmp);
            const double yAy = wg_dot(S, Ya, AYa, red, tmp);
            const double mu = yAy / yy;
            const double r2 = wg_combo(S, AYa, 1.0, Ya, -mu, nullptr, 0.0, red, tmp);
            if (threadIdx.x == 0) {
                mre[i] = mu;
                mim[i] = 0.0;
                res[i] = sqrt(r2) / sqrt(yy);
                yn[i] = sqrt(yy);
            }
        } else {
            const double* Yb = S.Y + (size_t)S.wcim[i] * S.ld;
            const double* AYb = S.AY + (size_t)S.wcim[i] * S.ld;
            const double aa = wg_dot(S, Ya, Ya, red, tmp);
            const double aAa = wg_dot(S, Ya, AYa, red, tmp);
            const double bb = wg_dot(S, Yb, Yb, red, tmp);
            const double bAb = wg_dot(S, Yb, AYb, red, tmp);
            const double aAb = wg_dot(S, Ya, AYb, red, tmp);
            const double bAa = wg_dot(S, Yb, AYa, red, tmp);
            const double yy = aa + bb;
            const double mr = (aAa + bAb) / yy, mi = (aAb - bAa) / yy;
            // A y - mu y, y = a + i b: real part A a - mr a + mi b,
            // imaginary part A b - mr b - mi a
            const double r1 = wg_combo(S, AYa, 1.0, Ya, -mr, Yb, mi, red, tmp);
            const double r2 = wg_combo(S, AYb, 1.0, Yb, -mr, Ya, -mi, red, tmp);
            if (threadIdx.x == 0) {
                mre[i] = mr;
                mim[i] = mi;
                res[i] = sqrt(r1 + r2) / sqrt(yy);
                yn[i] = sqrt(yy);
            }
        }
    }
    if (threadIdx.x == 0) S.j_done = S.j;
}

}  // namespace

// ---------------------------------------------------------------- host driver
namespace {

enum : int { ST_FREE = 0, ST_BUILD = 1, ST_CYCLE = 2, ST_TEST = 3, ST_DONE = 4, ST_RR = 5 };

struct BReqState {
    int state = ST_FREE;
    ppa_batch_request rq{};
    int64_t nnz = 0;
    double anorm = 0.0;
    int dmax = 0;
    // carved device pointers
    double *V = nullptr, *V2 = nullptr, *w = nullptr, *t1 = nullptr, *t2 = nullptr, *t3 = nullptr;
    double *H = nullptr, *Y = nullptr, *AY = nullptr, *Q = nullptr, *out = nullptr;
    double *rre = nullptr, *rim = nullptr;
    float* val32 = nullptr;   // mixed precision: FP32 values and chain vectors
    float *f1 = nullptr, *f2 = nullptr, *f3 = nullptr, *f4 = nullptr;
    int ld = 0, ldh = 0;
    // mixed precision: FP32 phase on, the pending test is the closing
    // Rayleigh-Ritz pass's
    bool f32 = false, rr_test = false;
    std::vector<double> hist;   // largest wanted residual per cycle
    int fp32_cycles = 0;
    int64_t passes32 = 0;
    // progress
    int j = 0, jend = 0, cycle = 0, deg = 0;
    int jstart = 0;   // first Krylov step of the current cycle (0, or kept vectors)
    bool init = false, restart = false;
    int qin = 0, qout = 0;
    std::vector<cplx> roots;
    RitzPlan plan;
    std::vector<double> Hm;
    int mc = 0;
    double hm_last = 0.0;
    bool broke = false;
    // results
    int status = PPA_OK;
    std::vector<cplx> mu;
    std::vector<double> res;
    std::vector<cplx> nu;
    int nconv = 0;
    int64_t mvps = 0, dots = 0, vops = 0;
    int build_status = PPA_OK;
    std::string err;
};

size_t carve_batch(Carver& c, int64_t n, int d, int m, int nev, int64_t nnz, bool mixed, BReqState* s) {
    const int cols = std::max(m, d) + 1;
    const int64_t ld = col_ld(n);
    double* V = c.take<double>((size_t)ld * cols);
    double* V2 = c.take<double>((size_t)ld * cols);
    double* w = c.take<double>((size_t)n);
    double* t1 = c.take<double>((size_t)n);
    double* t2 = c.take<double>((size_t)n);
    double* t3 = c.take<double>((size_t)n);
    double* H = c.take<double>((size_t)cols * (cols - 1));
    double* Y = c.take<double>((size_t)ld * 2 * nev);
    double* AY = c.take<double>((size_t)ld * 2 * nev);
    double* Q = c.take<double>((size_t)(m + 1) * std::max(m + 1, 2 * nev));
    double* out = c.take<double>(4 * BMAXW);
    double* rre = c.take<double>(std::max(d, 1));
    double* rim = c.take<double>(std::max(d, 1));
    float *v32 = nullptr, *f[4] = {nullptr, nullptr, nullptr, nullptr};
    if (mixed) {
        v32 = c.take<float>((size_t)std::max<int64_t>(nnz, 1));
        for (int i = 0; i < 4; ++i) f[i] = c.take<float>((size_t)n);
    }
    if (s) {
        s->V = V; s->V2 = V2; s->w = w; s->t1 = t1; s->t2 = t2; s->t3 = t3;
        s->H = H; s->Y = Y; s->AY = AY; s->Q = Q; s->out = out; s->rre = rre; s->rim = rim;
        s->val32 = v32;
        s->f1 = f[0]; s->f2 = f[1]; s->f3 = f[2]; s->f4 = f[3];
        s->ld = (int)ld;
        s->ldh = cols;
    }
    return c.bytes();
}

}  // namespace

struct Batch {
    int max_slots = 0;
    hipStream_t s = nullptr;
    std::vector<BReqState> st;
    std::vector<BSlot> desc;
    BSlot* ddesc = nullptr;
    int budget = 256;
};

static void batch_fill(BReqState& q, BSlot& d) {
    std::memset(&d, 0, sizeof(d));
    d.rowptr = q.rq.rowptr_d;
    d.colind = q.rq.colind_d;
    d.val = q.rq.val_d;
    d.V = q.V;
    d.V2 = q.V2;
    d.w = q.w;
    d.t1 = q.t1;
    d.t2 = q.t2;
    d.t3 = q.t3;
    d.H = q.H;
    d.Y = q.Y;
    d.AY = q.AY;
    d.Q = q.Q;
    d.out = q.out;
    d.rre = q.rre;
    d.rim = q.rim;
    d.val32 = q.val32;
    d.f1 = q.f1;
    d.f2 = q.f2;
    d.f3 = q.f3;
    d.f4 = q.f4;
    d.n = (int)q.rq.n;
    d.ld = q.ld;
    d.ldh = q.ldh;
    d.phase = PH_IDLE;
}

// harmonic Ritz values and Leja order from the downloaded GMRES Hessenberg
static void batch_finish_build(BReqState& q, hipStream_t s) {
    const int d = q.rq.d, ldh = q.ldh;
    std::vector<double> H((size_t)ldh * (ldh - 1));
    PPA_HIP(hipMemcpyAsync(H.data(), q.H, H.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    PPA_HIP(hipStreamSynchronize(s));
    int deff = d;
    for (int j = 0; j < d; ++j) {
        double colsq = 0.0;
        for (int i = 0; i <= j + 1; ++i) colsq += H[i + (size_t)j * ldh] * H[i + (size_t)j * ldh];
        if (!std::isfinite(colsq)) fail(PPA_ERR_NONFINITE, "batched GMRES: non-finite Hessenberg entry");
        if (H[j + 1 + (size_t)j * ldh] <= kBTol * std::sqrt(colsq)) {
            deff = j + 1;
            break;
        }
    }
    std::vector<double> Hb((size_t)(deff + 1) * deff, 0.0);
    for (int j = 0; j < deff; ++j)
        for (int i = 0; i <= std::min(j + 1, deff); ++i) {
            if (i == deff && deff < d) continue;
            Hb[i + (size_t)j * (deff + 1)] = H[i + (size_t)j * ldh];
        }
    if (deff < d) q.build_status = PPA_WARN_DEGREE_REDUCED;
    q.roots = leja_order(harmonic_ritz(deff, Hb));
    q.deg = (int)q.roots.size();
    std::vector<double> re(q.deg), im(q.deg);
    for (int i = 0; i < q.deg; ++i) {
        re[i] = q.roots[i].real();
        im[i] = q.roots[i].imag();
    }
    PPA_HIP(hipMemcpyAsync(q.rre, re.data(), q.deg * sizeof(double), hipMemcpyHostToDevice, s));
    PPA_HIP(hipMemcpyAsync(q.rim, im.data(), q.deg * sizeof(double), hipMemcpyHostToDevice, s));
    launch_zero(q.H, (int64_t)ldh * (ldh - 1), s);
    q.state = ST_CYCLE;
    q.j = 0;
    q.jstart = 0;
    q.jend = q.rq.m;
    q.init = true;
    q.restart = false;
    q.cycle = 1;
}

// Ritz pairs of H_m after a finished cycle: plan the test
static void batch_finish_cycle(BReqState& q, hipStream_t s) {
    const int m = q.rq.m, ldh = q.ldh;
    std::vector<double> H((size_t)ldh * (ldh - 1));
    PPA_HIP(hipMemcpyAsync(H.data(), q.H, H.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    PPA_HIP(hipStreamSynchronize(s));
    for (double x : H)
        if (!std::isfinite(x)) fail(PPA_ERR_NONFINITE, "batched Arnoldi: non-finite Hessenberg entry");
    // breakdown test on the columns built in this cycle (after a restart the
    // leading kept block is full, not Hessenberg)
    int mc = m;
    for (int j = q.jstart; j < m; ++j) {
        double colsq = 0.0;
        for (int i = 0; i <= j + 1; ++i) colsq += H[i + (size_t)j * ldh] * H[i + (size_t)j * ldh];
        if (H[j + 1 + (size_t)j * ldh] <= kBTol * std::sqrt(colsq)) {
            mc = j + 1;
            q.broke = true;
            break;
        }
    }
    q.mc = mc;
    q.Hm.assign((size_t)mc * mc, 0.0);
    for (int jj = 0; jj < mc; ++jj)
        for (int i = 0; i < mc; ++i) q.Hm[i + (size_t)jj * mc] = H[i + (size_t)jj * ldh];
    q.plan = plan_ritz(q.Hm, mc, q.rq.nev, 1.0);
    PPA_HIP(hipMemcpyAsync(q.Q, q.plan.Gw.data(), q.plan.Gw.size() * sizeof(double), hipMemcpyHostToDevice, s));
    q.qin = mc;
    q.qout = q.plan.ycols;
    q.hm_last = H[m + (size_t)(m - 1) * ldh];
    if (q.f32) ++q.fp32_cycles;
    q.state = ST_TEST;
}

// Closing FP64 Rayleigh-Ritz pass of a mixed-precision solve: K = V^T A V
// (downloaded from Q) and its Ritz pairs nearest the origin, tested next on
// A as every cycle's pairs are.
static void batch_finish_rr(BReqState& q, hipStream_t s) {
    const int J = q.qin;
    std::vector<double> K((size_t)J * J);
    PPA_HIP(hipMemcpyAsync(K.data(), q.Q, K.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    PPA_HIP(hipStreamSynchronize(s));
    for (double x : K)
        if (!std::isfinite(x)) fail(PPA_ERR_NONFINITE, "batched closing Rayleigh-Ritz: non-finite projection");
    q.mvps += J;
    q.dots += (int64_t)J * J;
    q.plan = plan_ritz(K, J, q.rq.nev, 0.0);
    PPA_HIP(hipMemcpyAsync(q.Q, q.plan.Gw.data(), q.plan.Gw.size() * sizeof(double), hipMemcpyHostToDevice, s));
    q.qin = J;
    q.qout = q.plan.ycols;
    q.rr_test = true;
    q.state = ST_TEST;
}


// Rayleigh quotients and residuals of a finished test: finish the solve or
// plan the thick restart.  Returns true when the solve is done.
static bool batch_finish_test(BReqState& q, hipStream_t s) {
    double out[4 * BMAXW];
    PPA_HIP(hipMemcpyAsync(out, q.out, sizeof(out), hipMemcpyDeviceToHost, s));
    PPA_HIP(hipStreamSynchronize(s));
    const RitzPlan& R = q.plan;
    const int nw = R.nw, nev = q.rq.nev, m = q.rq.m;
    std::vector<cplx> mu(nw);
    std::vector<double> res(nw);
    double mx = 0.0;
    for (int i = 0; i < nw; ++i) {
        mu[i] = cplx(out[i], out[BMAXW + i]);
        res[i] = out[2 * BMAXW + i];
        if (!std::isfinite(res[i]) || !std::isfinite(mu[i].real()))
            fail(PPA_ERR_NONFINITE, "batched Ritz test: non-finite result");
        mx = std::max(mx, res[i]);
    }
    q.mvps += ritz_mvps(R);
    const double rtol_abs = q.rq.rtol * q.anorm;
    const bool conv = nw == nev && mx <= rtol_abs;
    if (q.rr_test) {
        // the closing Rayleigh-Ritz pass: done if all wanted pairs meet rtol,
        // else FP64 cycles from the start vector again (as in the
        // single-solve driver)
        q.rr_test = false;
        q.hist.back() = std::min(q.hist.back(), mx);
        if (!conv) {
            launch_zero(q.H, (int64_t)q.ldh * (q.ldh - 1), s);
            PPA_HIP(hipStreamSynchronize(s));
            q.restart = false;
            q.init = true;
            q.j = 0;
            q.jstart = 0;
            q.jend = m;
            q.cycle += 1;
            q.state = ST_CYCLE;
            return false;
        }
    } else {
        q.hist.push_back(mx);
    }
    if (conv || q.broke || q.cycle >= q.rq.max_cycles) {
        q.mu = mu;
        q.res = res;
        q.nu.assign(R.nu.begin(), R.nu.begin() + nw);
        q.nconv = 0;
        for (int i = 0; i < nw; ++i) q.nconv += res[i] <= rtol_abs;
        q.status = conv ? PPA_OK : (q.broke ? PPA_WARN_BREAKDOWN : PPA_WARN_NOT_CONVERGED);
        q.state = ST_DONE;
        return true;
    }
    if (q.f32 && leave_fp32(q.hist, q.anorm)) {
        // leave the FP32 phase: closing Rayleigh-Ritz with A on the m + 1
        // basis vectors the FP32 cycle built
        q.f32 = false;
        q.qin = q.mc + 1;
        q.state = ST_RR;
        return false;
    }
    const RestartPlan RP = plan_restart(R, q.Hm, q.hm_last, m, q.rq.k);
    PPA_HIP(hipMemcpyAsync(q.Q, RP.Qp.data(), RP.Qp.size() * sizeof(double), hipMemcpyHostToDevice, s));
    std::vector<double> Hn((size_t)q.ldh * (q.ldh - 1), 0.0);
    for (int jj = 0; jj < m; ++jj)
        for (int i = 0; i <= m; ++i) Hn[i + (size_t)jj * q.ldh] = RP.Hn[i + (size_t)jj * (m + 1)];
    PPA_HIP(hipMemcpyAsync(q.H, Hn.data(), Hn.size() * sizeof(double), hipMemcpyHostToDevice, s));
    PPA_HIP(hipStreamSynchronize(s));
    q.qin = m + 1;
    q.qout = RP.kk + 1;
    q.restart = true;
    q.init = false;
    q.j = RP.kk;
    q.jstart = RP.kk;
    q.jend = m;
    q.cycle += 1;
    q.state = ST_CYCLE;
    return false;
}

__global__ void k_absrowmax(const int32_t* __restrict__ rowptr, const double* __restrict__ val, int n,
                            double* __restrict__ out) {
    __shared__ double sm[BWG];
    double mx = 0.0;
    for (int r = threadIdx.x; r < n; r += BWG) {
        double s = 0.0;
        for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) s += fabs(val[k]);
        mx = fmax(mx, s);
    }
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int w = BWG / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sm[0];
}

size_t batch_ws_bytes(int64_t n, int d, int m, int nev, int64_t nnz, int precision) {
    Carver c(nullptr, 0);
    return carve_batch(c, n, d, m, nev, nnz, precision == PPA_MIXED, nullptr);
}

Batch* batch_create(int max_slots, hipStream_t s) {
    PPA_REQUIRE(max_slots >= 1 && max_slots <= 65536, "max_slots out of range");
    Batch* B = new Batch();
    B->max_slots = max_slots;
    B->s = s;
    B->st.resize(max_slots);
    B->desc.resize(max_slots);
    if (hipMalloc(&B->ddesc, (size_t)max_slots * sizeof(BSlot)) != hipSuccess) {
        delete B;
        fail(PPA_ERR_HIP, "batch: device descriptor allocation failed");
    }
    return B;
}

void batch_destroy(Batch* B) {
    if (!B) return;
    (void)hipFree(B->ddesc);
    delete B;
}

int batch_submit(Batch& B, const ppa_batch_request& rq, int* slot, int precision) {
    PPA_REQUIRE(precision == PPA_F64 || precision == PPA_MIXED, "batch: precision must be F64 or MIXED");
    PPA_REQUIRE(rq.n >= 1 && rq.n < (int64_t(1) << 31), "batch: n out of range");
    PPA_REQUIRE(rq.rowptr_d && rq.colind_d && rq.val_d && rq.b_d && rq.v0_d && rq.ws_d,
                "batch: matrix, start vectors and workspace are required");
    PPA_REQUIRE(rq.d >= 1 && rq.d <= BMAXJ - 2, "batch: degree out of range");
    PPA_REQUIRE(rq.m >= 2 && rq.m <= 64 && rq.nev >= 1 && rq.nev <= rq.k && rq.k < rq.m && rq.nev <= BMAXW,
                "batch: need 1 <= nev <= k < m <= 64, nev <= 32");
    PPA_REQUIRE(rq.n > rq.m && rq.n > rq.d, "batch: n must exceed m and d");
    PPA_REQUIRE(rq.max_cycles >= 1 && rq.rtol > 0.0, "batch: max_cycles >= 1 and rtol > 0");
    int free_slot = -1;
    for (int i = 0; i < B.max_slots; ++i)
        if (B.st[i].state == ST_FREE) {
            free_slot = i;
            break;
        }
    if (free_slot < 0) {
        *slot = -1;
        fail(PPA_ERR_BUSY, "batch: no free slot");
    }
    BReqState q;
    q.rq = rq;
    const bool mixed = precision == PPA_MIXED;
    int32_t nnz = 0;
    if (mixed) {
        PPA_HIP(hipMemcpyAsync(&nnz, rq.rowptr_d + rq.n, sizeof(int32_t), hipMemcpyDeviceToHost, B.s));
        PPA_HIP(hipStreamSynchronize(B.s));
        PPA_REQUIRE(nnz >= 0, "batch: negative nonzero count");
    }
    Carver c(rq.ws_d, rq.ws_bytes);
    carve_batch(c, rq.n, rq.d, rq.m, rq.nev, nnz, mixed, &q);
    c.check();
    if (mixed) {
        launch_cast_f64_f32(rq.val_d, q.val32, nnz, B.s);
        q.f32 = true;
    }
    // ||A||_inf (one small reduction) unless given
    if (rq.anorm > 0.0) {
        q.anorm = rq.anorm;
    } else {
        hipLaunchKernelGGL(k_absrowmax, dim3(1), dim3(BWG), 0, B.s, rq.rowptr_d, rq.val_d, (int)rq.n, q.out);
        PPA_HIP(hipGetLastError());
        PPA_HIP(hipMemcpyAsync(&q.anorm, q.out, sizeof(double), hipMemcpyDeviceToHost, B.s));
        PPA_HIP(hipStreamSynchronize(B.s));
    }
    launch_zero(q.H, (int64_t)q.ldh * (q.ldh - 1), B.s);
    q.state = ST_BUILD;
    q.j = 0;
    q.jend = rq.d;
    q.init = true;
    B.st[free_slot] = std::move(q);
    *slot = free_slot;
    return PPA_OK;
}

int batch_step(Batch& B, int* finished, int cap, int* nfin, int* nactive) {
    std::vector<int> act;
    for (int i = 0; i < B.max_slots; ++i) {
        const int st = B.st[i].state;
        if (st == ST_BUILD || st == ST_CYCLE || st == ST_TEST || st == ST_RR) act.push_back(i);
    }
    *nfin = 0;
    if (nactive) *nactive = (int)act.size();
    if (act.empty()) return PPA_OK;
    for (size_t a = 0; a < act.size(); ++a) {
        BReqState& q = B.st[act[a]];
        BSlot& d = B.desc[a];
        batch_fill(q, d);
        d.j = q.j;
        d.budget = B.budget;
        if (q.state == ST_BUILD) {
            d.phase = PH_BUILD;
            d.use_poly = 0;
            d.init = q.j == 0;
            d.start = q.rq.b_d;
            d.jend = q.rq.d;
        } else if (q.state == ST_CYCLE) {
            d.phase = PH_CYCLE;
            d.use_poly = 1;
            d.deg = q.deg;
            d.init = q.init;
            d.start = q.rq.v0_d;
            d.restart = q.restart;
            d.f32 = q.f32;
            d.qin = q.qin;
            d.qout = q.qout;
            d.jend = q.jend;
        } else if (q.state == ST_RR) {
            d.phase = PH_RR;
            d.qin = q.qin;
        } else {
            d.phase = PH_TEST;
            d.qin = q.qin;
            d.qout = q.qout;
            d.nw = q.plan.nw;
            d.ycols = q.plan.ycols;
            for (int i = 0; i < q.plan.nw; ++i) {
                d.wcre[i] = q.plan.cre[i];
                d.wcim[i] = q.plan.cim[i];
                d.wdup[i] = q.plan.dup[i];
            }
        }
    }
    const size_t nb = act.size();
    PPA_HIP(hipMemcpyAsync(B.ddesc, B.desc.data(), nb * sizeof(BSlot), hipMemcpyHostToDevice, B.s));
    hipLaunchKernelGGL(k_batch, dim3((unsigned)nb), dim3(BWG), 0, B.s, B.ddesc);
    PPA_HIP(hipGetLastError());
    std::vector<BSlot> back(nb);
    PPA_HIP(hipMemcpyAsync(back.data(), B.ddesc, nb * sizeof(BSlot), hipMemcpyDeviceToHost, B.s));
    PPA_HIP(hipStreamSynchronize(B.s));
    int nf = 0;
    for (size_t a = 0; a < nb; ++a) {
        const int slot = act[a];
        BReqState& q = B.st[slot];
        try {
            const int jd = back[a].j_done;
            if (q.state == ST_BUILD) {
                q.j = jd;
                if (q.j >= q.rq.d) batch_finish_build(q, B.s);
            } else if (q.state == ST_CYCLE) {
                const int op = q.deg;
                for (int jj = q.j; jj < jd; ++jj) {
                    q.mvps += op;
                    q.vops += op + 4 * (jj + 1) + 2;
                    q.dots += 2 * (jj + 1) + 1;
                    if (q.f32) q.passes32 += op;
                }
                if (q.restart) {
                    std::swap(q.V, q.V2);
                    q.restart = false;
                }
                q.init = false;
                q.j = jd;
                if (q.j >= q.jend) batch_finish_cycle(q, B.s);
            } else if (q.state == ST_RR) {
                batch_finish_rr(q, B.s);
            } else {
                if (batch_finish_test(q, B.s)) {
                    if (nf < cap && finished) finished[nf] = slot;
                    ++nf;
                }
            }
        } catch (const Error& e) {
            q.status = e.code;
            q.err = e.what();
            q.state = ST_DONE;
            if (nf < cap && finished) finished[nf] = slot;
            ++nf;
        }
    }
    *nfin = nf;
    return PPA_OK;
}

int batch_result(Batch& B, int slot, ppa_eigs_result& r) {
    PPA_REQUIRE(slot >= 0 && slot < B.max_slots, "batch: slot out of range");
    BReqState& q = B.st[slot];
    PPA_REQUIRE(q.state == ST_DONE, "batch: slot %d has no finished solve", slot);
    PPA_REQUIRE(r.lam_re && r.lam_im && r.resid, "batch: result arrays are required");
    const int status = q.status;
    if (status < 0) {
        const std::string msg = q.err;
        B.st[slot] = BReqState();
        fail(status, "%s", msg.c_str());
    }
    {
        const int nw = (int)q.mu.size(), nev = q.rq.nev;
        std::vector<int> ord(nw);
        for (int i = 0; i < nw; ++i) ord[i] = i;
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
            const double ma = std::abs(q.mu[a]), mb = std::abs(q.mu[b]);
            if (ma != mb) return ma < mb;
            if (q.mu[a].real() != q.mu[b].real()) return q.mu[a].real() < q.mu[b].real();
            return q.mu[a].imag() < q.mu[b].imag();
        });
        double mx = 0.0;
        for (int t = 0; t < nev; ++t) {
            if (t < nw) {
                const int i = ord[t];
                r.lam_re[t] = q.mu[i].real();
                r.lam_im[t] = q.mu[i].imag();
                r.resid[t] = q.res[i];
                if (r.ritz_re) r.ritz_re[t] = q.nu[i].real();
                if (r.ritz_im) r.ritz_im[t] = q.nu[i].imag();
                mx = std::max(mx, q.res[i]);
            } else {
                r.lam_re[t] = r.lam_im[t] = r.resid[t] = std::nan("");
            }
        }
        r.nconv = q.nconv;
        r.cycles = q.cycle;
        r.mvps = q.mvps;
        r.dots = q.dots;
        r.vops = q.vops;
        r.max_resid = mx;
        r.fp32_cycles = q.fp32_cycles;
        r.spmv_passes = q.mvps;
        r.spmv_passes_f32 = q.passes32;
        r.t_apply_ms = r.t_cgs_ms = 0.0;
    }
    B.st[slot] = BReqState();
    return status;
}

}  // namespace ppa
