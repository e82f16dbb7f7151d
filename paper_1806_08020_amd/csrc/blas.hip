// Dense kernels around the polynomial operator: classical Gram-Schmidt with
// one reorthogonalisation pass against the Krylov basis V (section 4), the
// tall-skinny product V Q of the thick restart and of the Ritz vectors on
// FP64 MFMA, and small deterministic reductions for the convergence test.
//
// V is column-major (one Krylov vector per column, leading dimension a
// multiple of 32 doubles).  Tall-skinny V^T w products are two-stage: each
// block reduces its contiguous row range (wavefront shuffles, then LDS across
// the 4 waves) into a partial per column, and a second kernel sums the
// partials of a column in a fixed tree.  No floating-point atomics are used,
// so every result is bitwise reproducible run to run.
#include "ppa_internal.hpp"

#include <initializer_list>

#include <algorithm>
#include <type_traits>
#include <utility>
#include <cmath>

namespace ppa {

namespace {

constexpr int BS = 256;
constexpr int NW = BS / 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Reduce `count` per-thread values acc[0..count) across the block and write
// lane results to dst[c * stride] for c < count (thread c does column c).
template <int NC>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NC], int count, double* red,
                                                   double* dst, int64_t stride) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (c < count) {
            const double v = wave_sum(acc[c]);
            if (lane == 0) red[w * NC + c] = v;
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < count; c += BS) {
        double t = 0.0;
        for (int q = 0; q < NW; ++q) t += red[q * NC + c];
        dst[c * stride] = t;
    }
}

struct RowRange {
    int64_t beg, end;
};
// contiguous row range of block blockIdx.x when n rows are split over nb blocks
__device__ __forceinline__ RowRange rows_of_block(int64_t n, int nb) {
    const int64_t per = (n + nb - 1) / nb;
    const int64_t beg = (int64_t)blockIdx.x * per;
    return {beg, min(n, beg + per)};
}

// Row mapping of the streaming kernels: block b owns rows
// [b * BS * RPT, (b + 1) * BS * RPT); thread t handles rows base + t + i * BS.
// Rows past n are clamped to n - 1 for loads (always in bounds) and carry a
// zero weight, so every load can be issued unconditionally.
#ifndef PPA_CGS_RPT
#define PPA_CGS_RPT 8
#endif
#ifndef PPA_CGS_CT
#define PPA_CGS_CT 8
#endif
constexpr int RPT = PPA_CGS_RPT;   // rows per thread
constexpr int CT = PPA_CGS_CT;     // column tile of the projection

// partial[c * nb + b] = sum over the block's rows of V[c][r] w[r] (c < j),
// and partial[j * nb + b] = sum w[r]^2 when with_norm.
__global__ __launch_bounds__(BS) void k_proj(const double* __restrict__ V, int64_t ldv, int64_t n,
                                             int j, const double* __restrict__ w,
                                             double* __restrict__ partial, int nb, int with_norm) {
    __shared__ double red[NW * CT];
    const int64_t base = (int64_t)blockIdx.x * BS * RPT + threadIdx.x;
    double wr[RPT];
    int64_t rr[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int64_t r = base + (int64_t)i * BS;
        rr[i] = r < n ? r : n - 1;
        wr[i] = r < n ? w[rr[i]] : 0.0;
    }
    if (with_norm) {
        double a[1] = {0.0};
#pragma unroll
        for (int i = 0; i < RPT; ++i) a[0] += wr[i] * wr[i];
        block_reduce_store<1>(a, 1, red, partial + (int64_t)j * nb + blockIdx.x, nb);
        __syncthreads();
    }
    for (int c0 = 0; c0 < j; c0 += CT) {
        double acc[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[c] = 0.0;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const double* col = V + (int64_t)min(c0 + c, j - 1) * ldv;
#pragma unroll
            for (int i = 0; i < RPT; ++i) acc[c] += col[rr[i]] * wr[i];
        }
        block_reduce_store<CT>(acc, min(CT, j - c0), red, partial + (int64_t)c0 * nb + blockIdx.x, nb);
        __syncthreads();
    }
}

// k_proj on row pairs: thread t of block b reads rows r, r + 1 with
// r = b * BS * RPT + 2 t + 2 i BS (i < RPT / 2) as one 16-byte load per
// column.  For even n, 16-byte aligned V and w and even ldv; pairs past n
// re-read the last pair with weight zero.
__global__ __launch_bounds__(BS) void k_proj2(const double* __restrict__ V, int64_t ldv, int64_t n,
                                              int j, const double* __restrict__ w,
                                              double* __restrict__ partial, int nb, int with_norm) {
    constexpr int RP = RPT / 2;
    __shared__ double red[NW * CT];
    const int64_t base = (int64_t)blockIdx.x * BS * RPT + 2 * threadIdx.x;
    double2 wr[RP];
    int64_t rr[RP];
#pragma unroll
    for (int i = 0; i < RP; ++i) {
        const int64_t r = base + (int64_t)i * 2 * BS;
        rr[i] = r < n ? r : n - 2;
        const double2 v = *reinterpret_cast<const double2*>(w + rr[i]);
        wr[i] = r < n ? v : make_double2(0.0, 0.0);
    }
    if (with_norm) {
        double a[1] = {0.0};
#pragma unroll
        for (int i = 0; i < RP; ++i) {
            a[0] += wr[i].x * wr[i].x;
            a[0] += wr[i].y * wr[i].y;
        }
        block_reduce_store<1>(a, 1, red, partial + (int64_t)j * nb + blockIdx.x, nb);
        __syncthreads();
    }
    for (int c0 = 0; c0 < j; c0 += CT) {
        double acc[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[c] = 0.0;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const double* col = V + (int64_t)min(c0 + c, j - 1) * ldv;
#pragma unroll
            for (int i = 0; i < RP; ++i) {
                const double2 v = *reinterpret_cast<const double2*>(col + rr[i]);
                acc[c] += v.x * wr[i].x;
                acc[c] += v.y * wr[i].y;
            }
        }
        block_reduce_store<CT>(acc, min(CT, j - c0), red, partial + (int64_t)c0 * nb + blockIdx.x, nb);
        __syncthreads();
    }
}

// out = t - V h (h of length j, device); partial[b] = ||out||^2 over the
// block's rows when partial is non-null.  out may equal t.
__global__ __launch_bounds__(BS) void k_update(const double* __restrict__ V, int64_t ldv, int64_t n,
                                               int j, const double* __restrict__ h,
                                               const double* t, double* out,
                                               double* __restrict__ partial, int nb) {
    __shared__ double hs[CGS_JMAX_ALL + 8];
    __shared__ double red[NW];
    for (int c = threadIdx.x; c < CGS_JMAX_ALL + 8; c += BS) hs[c] = c < j ? h[c] : 0.0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * BS * RPT + threadIdx.x;
    double tv[RPT];
    int64_t rr[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int64_t r = base + (int64_t)i * BS;
        rr[i] = r < n ? r : n - 1;
        tv[i] = t[rr[i]];
    }
    for (int c0 = 0; c0 < j; c0 += 8) {
        double v[8][RPT];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const double* col = V + (int64_t)min(c0 + c, j - 1) * ldv;
#pragma unroll
            for (int i = 0; i < RPT; ++i) v[c][i] = col[rr[i]];
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const double hc = hs[c0 + c];
#pragma unroll
            for (int i = 0; i < RPT; ++i) tv[i] -= v[c][i] * hc;
        }
    }
    double nrm = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        if (base + (int64_t)i * BS < n) {
            out[rr[i]] = tv[i];
            nrm += tv[i] * tv[i];
        }
    }
    if (partial) {
        double acc[1] = {nrm};
        block_reduce_store<1>(acc, 1, red, partial + blockIdx.x, nb);
    }
}

// f(integral_constant<int, I>) for I = 0..N-1, each index a compile-time constant.
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// One butterfly reduce-scatter step and the ones after it: a lane keeps half
// of its K columns (the upper half when bit O of its lane is set) and adds
// the partner lane's copy of that half.
template <int JT, int K, int O>
__device__ __forceinline__ void butterfly(double (&v)[JT], int lane, int& col) {
    if constexpr (K > 1) {
        const bool up = (lane & O) != 0;
        static_for<K / 2>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const double send = up ? v[i] : v[K / 2 + i];
            const double keep = up ? v[K / 2 + i] : v[i];
            v[i] = keep + __shfl_xor(send, O, 64);
        });
        if (up) col += K / 2;
        butterfly<JT, K / 2, O / 2>(v, lane, col);
    }
}

// The reorthogonalisation's update and projection in one pass over V:
//   t = w - V h          (h = the first projection, length j)
//   partial[c * nb + b] = sum over the block's rows of V[c][r] t[r]  (c < j)
// One row per thread; its JT >= j entries of V stay in registers between the
// two steps.  The column sums of a wave are formed by a butterfly
// reduce-scatter: at each step a lane keeps half of its columns and adds the
// partner's copy of that half, so a wave needs about JT shuffles instead of
// 6 per column; lane l then holds the wave's sum for one column.  The four
// waves are combined through LDS in a fixed order.
template <int JT>
__global__ __launch_bounds__(BS) void k_update_proj(const double* __restrict__ V, int64_t ldv,
                                                    int64_t n, int j, const double* __restrict__ h,
                                                    const double* __restrict__ w,
                                                    double* __restrict__ t,
                                                    double* __restrict__ partial, int nb) {
    static_assert(JT >= 1 && JT <= 64 && (JT & (JT - 1)) == 0, "JT: power of two up to 64");
    __shared__ double hs[JT];
    __shared__ double red[NW][JT];
    const int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x;
    const int64_t rr = r < n ? r : n - 1;
    // columns past j re-read column j - 1 (weight 0): unconditional loads
    // keep the register count lowest; the instance is chosen with JT < 2j
    // every index into v is a compile-time constant (static_for), so the
    // array lives in registers from the start; loop-indexed accesses let the
    // compiler turn the butterfly's selects into dynamically indexed
    // register reads (long compare-and-select chains) for some JT
    double v[JT];
    static_for<JT>([&](auto ic) {
        constexpr int c = decltype(ic)::value;
        v[c] = V[(int64_t)min(c, j - 1) * ldv + rr];
    });
    double tv = w[rr];
    // h is staged in LDS after the row's loads are in flight
    for (int c = threadIdx.x; c < JT; c += BS) hs[c] = c < j ? h[c] : 0.0;
    __syncthreads();
    static_for<JT>([&](auto ic) {
        constexpr int c = decltype(ic)::value;
        tv -= v[c] * hs[c];
    });
    if (r < n) t[r] = tv;
    const double wt = r < n ? tv : 0.0;
    static_for<JT>([&](auto ic) {
        constexpr int c = decltype(ic)::value;
        v[c] = c < j ? v[c] * wt : 0.0;
    });
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int col = 0;
    butterfly<JT, JT, 32>(v, lane, col);
    // lanes that share a column now hold partial sums over disjoint lanes
    for (int o = 32 / JT; o > 0; o >>= 1) v[0] += __shfl_xor(v[0], o, 64);
    if ((lane & (64 / JT - 1)) == 0) red[wave][col] = v[0];
    __syncthreads();
    for (int c = threadIdx.x; c < j; c += BS) {
        double s = 0.0;
        for (int q = 0; q < NW; ++q) s += red[q][c];
        partial[(int64_t)c * nb + blockIdx.x] = s;
    }
}

// k_update_proj for JH < j <= 2 JH with half the registers: a block covers
// BS / 2 rows; waves 0 and 1 hold the columns 0 .. JH - 1 of those rows,
// waves 2 and 3 the columns JH .. 2 JH - 1 (the half is uniform in a wave, so
// column addresses stay scalar).  Each lane sums its half of V h, the halves
// meet in LDS, and the row's update is (w - s_0) - s_1 on both sides.
template <int JH>
__global__ __launch_bounds__(BS) void k_update_proj_halves(const double* __restrict__ V, int64_t ldv,
                                                           int64_t n, int j,
                                                           const double* __restrict__ h,
                                                           const double* __restrict__ w,
                                                           double* __restrict__ t,
                                                           double* __restrict__ partial, int nb) {
    static_assert(BS == 256, "two waves per half");
    static_assert(JH == 16 || JH == 32, "JH: 16 or 32");
    __shared__ double hs[2 * JH];
    __shared__ double sx[BS];
    __shared__ double red[NW][JH];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int half = wave >> 1;
    const int64_t r = (int64_t)blockIdx.x * (BS / 2) + (wave & 1) * 64 + lane;
    const int64_t rr = r < n ? r : n - 1;
    double v[JH];
    static_for<JH>([&](auto ic) {
        constexpr int c = decltype(ic)::value;
        v[c] = V[(int64_t)min(JH * half + c, j - 1) * ldv + rr];
    });
    const double tw = w[rr];
    for (int c = threadIdx.x; c < 2 * JH; c += BS) hs[c] = c < j ? h[c] : 0.0;
    __syncthreads();
    double sp = 0.0;
    static_for<JH>([&](auto ic) {
        constexpr int c = decltype(ic)::value;
        sp += v[c] * hs[JH * half + c];
    });
    sx[threadIdx.x] = sp;
    __syncthreads();
    const double so = sx[threadIdx.x ^ 128];
    const double tv = (tw - (half ? so : sp)) - (half ? sp : so);
    if (half == 0 && r < n) t[r] = tv;
    const double wt = r < n ? tv : 0.0;
    static_for<JH>([&](auto ic) {
        constexpr int c = decltype(ic)::value;
        v[c] = JH * half + c < j ? v[c] * wt : 0.0;
    });
    int col = 0;
    butterfly<JH, JH, 32>(v, lane, col);
    // lanes that share a column hold partial sums over disjoint lanes
    for (int o = 32 / JH; o > 0; o >>= 1) v[0] += __shfl_xor(v[0], o, 64);
    if ((lane & (64 / JH - 1)) == 0) red[wave][col] = v[0];
    __syncthreads();
    for (int c = threadIdx.x; c < j; c += BS) {
        const double s = c < JH ? red[0][c] + red[1][c] : red[2][c - JH] + red[3][c - JH];
        partial[(int64_t)c * nb + blockIdx.x] = s;
    }
}

// out[c] = sum_b partial[c * nb + b], one block per column, fixed tree.
// Each thread sums its strided share in order, eight loads in flight at a time.
__global__ __launch_bounds__(BS) void k_reduce_cols(const double* __restrict__ partial, int nb,
                                                    double* __restrict__ out) {
    __shared__ double red[NW];
    const double* p = partial + (int64_t)blockIdx.x * nb;
    double s = 0.0;
    int b = threadIdx.x;
    for (; b + 7 * BS < nb; b += 8 * BS) {
        double a[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = p[b + i * BS];
#pragma unroll
        for (int i = 0; i < 8; ++i) s += a[i];
    }
    for (; b < nb; b += BS) s += p[b];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < NW; ++q) t += red[q];
        out[blockIdx.x] = t;
    }
}

// Hessenberg column: H[i] = h1[i] + h2[i] (i < j), H[j] = beta = ||w_out||;
// h1[j] holds ||w_in||^2 and scal[1] ||w_out||^2.  scal[0] = ||w_in||^2,
// scal[2] = 1/beta, or 0 when beta <= tol * ||w_in|| (breakdown).
__global__ void k_cgs_finalize(const double* __restrict__ h1, const double* __restrict__ h2,
                               int j, double* __restrict__ scal, double* __restrict__ Hcol,
                               double tol) {
    for (int i = threadIdx.x; i < j; i += blockDim.x) Hcol[i] = h1[i] + h2[i];
    if (threadIdx.x == 0) {
        const double beta = sqrt(scal[1]);
        scal[0] = h1[j];
        const double w0 = sqrt(h1[j]);
        Hcol[j] = beta;
        scal[2] = (beta > tol * w0 && beta > 0.0) ? 1.0 / beta : 0.0;
    }
}

// k_update on row pairs (same mapping and conditions as k_proj2; t and out
// 16-byte aligned).
__global__ __launch_bounds__(BS) void k_update2(const double* __restrict__ V, int64_t ldv, int64_t n,
                                                int j, const double* __restrict__ h,
                                                const double* t, double* out,
                                                double* __restrict__ partial, int nb) {
    constexpr int RP = RPT / 2;
    __shared__ double hs[CGS_JMAX_ALL + 8];
    __shared__ double red[NW];
    for (int c = threadIdx.x; c < CGS_JMAX_ALL + 8; c += BS) hs[c] = c < j ? h[c] : 0.0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * BS * RPT + 2 * threadIdx.x;
    double2 tv[RP];
    int64_t rr[RP];
#pragma unroll
    for (int i = 0; i < RP; ++i) {
        const int64_t r = base + (int64_t)i * 2 * BS;
        rr[i] = r < n ? r : n - 2;
        tv[i] = *reinterpret_cast<const double2*>(t + rr[i]);
    }
    for (int c0 = 0; c0 < j; c0 += 8) {
        double2 v[8][RP];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const double* col = V + (int64_t)min(c0 + c, j - 1) * ldv;
#pragma unroll
            for (int i = 0; i < RP; ++i) v[c][i] = *reinterpret_cast<const double2*>(col + rr[i]);
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const double hc = hs[c0 + c];
#pragma unroll
            for (int i = 0; i < RP; ++i) {
                tv[i].x -= v[c][i].x * hc;
                tv[i].y -= v[c][i].y * hc;
            }
        }
    }
    double nrm = 0.0;
#pragma unroll
    for (int i = 0; i < RP; ++i) {
        if (base + (int64_t)i * 2 * BS < n) {
            *reinterpret_cast<double2*>(out + rr[i]) = tv[i];
            nrm += tv[i].x * tv[i].x;
            nrm += tv[i].y * tv[i].y;
        }
    }
    if (partial) {
        double acc[1] = {nrm};
        block_reduce_store<1>(acc, 1, red, partial + blockIdx.x, nb);
    }
}

// k_reduce_cols on the one column of ||w_out||^2 partials, k_cgs_finalize
// and v_next = w_out * scal[2] in one launch: every block sums the partials
// in k_reduce_cols' order (so all blocks, and the separate launches, get the
// same bits), block 0 writes the Hessenberg column and scal, and each block
// scales its share of w_out into v_next.
__global__ __launch_bounds__(BS) void k_finalize_scale(const double* __restrict__ partial, int nb,
                                                       const double* __restrict__ h1,
                                                       const double* __restrict__ h2, int j,
                                                       double* __restrict__ scal,
                                                       double* __restrict__ Hcol, double tol,
                                                       const double* __restrict__ w_out,
                                                       double* __restrict__ v_next, int64_t n) {
    __shared__ double red[NW];
    __shared__ double inv_s;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += BS) s += partial[b];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < NW; ++q) t += red[q];
        const double beta = sqrt(t);
        const double w0 = sqrt(h1[j]);
        const double inv = (beta > tol * w0 && beta > 0.0) ? 1.0 / beta : 0.0;
        inv_s = inv;
        if (blockIdx.x == 0) {
            scal[0] = h1[j];
            scal[1] = t;
            scal[2] = inv;
            Hcol[j] = beta;
        }
    }
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < j; i += BS) Hcol[i] = h1[i] + h2[i];
    __syncthreads();
    const double inv = inv_s;
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
        v_next[i] = w_out[i] * inv;
}

// ---------------------------------------------------------------- delayed form
// partial columns (stride nb): [0, jq) Q^T u, [jq, 2 jq) Q^T w, then u.u,
// u.w, w.w over the block's rows; a null u or w counts as zero.
__global__ __launch_bounds__(BS) void k_dproj(const double* __restrict__ V, int64_t ldv, int64_t n,
                                              int jq, const double* __restrict__ u,
                                              const double* __restrict__ w,
                                              double* __restrict__ partial, int nb) {
    constexpr int CH = CT / 2;   // columns per tile (two products each)
    __shared__ double red[NW * CT];
    const int64_t base = (int64_t)blockIdx.x * BS * RPT + threadIdx.x;
    double ur[RPT], wr[RPT];
    int64_t rr[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int64_t r = base + (int64_t)i * BS;
        rr[i] = r < n ? r : n - 1;
        ur[i] = (u && r < n) ? u[rr[i]] : 0.0;
        wr[i] = (w && r < n) ? w[rr[i]] : 0.0;
    }
    {
        double sc[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            sc[0] += ur[i] * ur[i];
            sc[1] += ur[i] * wr[i];
            sc[2] += wr[i] * wr[i];
        }
        block_reduce_store<3>(sc, 3, red, partial + (int64_t)(2 * jq) * nb + blockIdx.x, nb);
        __syncthreads();
    }
    for (int c0 = 0; c0 < jq; c0 += CH) {
        double acc[2 * CH];
#pragma unroll
        for (int c = 0; c < 2 * CH; ++c) acc[c] = 0.0;
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const double* col = V + (int64_t)min(c0 + c, jq - 1) * ldv;
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const double v = col[rr[i]];
                acc[c] += v * ur[i];
                acc[CH + c] += v * wr[i];
            }
        }
        const int cnt = min(CH, jq - c0);
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
        for (int c = 0; c < 2 * CH; ++c) {
            if ((c % CH) < cnt) {
                const double v = wave_sum(acc[c]);
                if (lane == 0) red[wv * CT + c] = v;
            }
        }
        __syncthreads();
        for (int c = threadIdx.x; c < 2 * CH; c += BS) {
            if ((c % CH) >= cnt) continue;
            double t = 0.0;
            for (int q = 0; q < NW; ++q) t += red[q * CT + c];
            const int col = c < CH ? c0 + c : jq + c0 + (c - CH);
            partial[(int64_t)col * nb + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

// Coefficients of one delayed step from the reduced inner products dred
// (layout of k_dproj) and the device Hessenberg matrix; one block.
// coef: a [0, JMAX), g [JMAX, 2 JMAX), then 1/beta, the scale of w, gamma.
__global__ __launch_bounds__(BS) void k_dcoef(int kind, int jq, const double* __restrict__ dred,
                                              double* __restrict__ Hd, int64_t ldh,
                                              double* __restrict__ coef, double* __restrict__ scal,
                                              double tol) {
    __shared__ double sa[CGS_JMAX_ALL], sc[CGS_JMAX_ALL + 1];
    __shared__ double rsum[NW * 2];
    __shared__ double s_inv, s_gamma;
    double* g = coef + CGS_JMAX_ALL;
    double* sv = coef + 2 * CGS_JMAX_ALL;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (kind == DCGS_FIRST) {
        // h = Q^T z: provisional column jq - 1; u_out = z - Q h
        double hs = 0.0;
        for (int i = tid; i < jq; i += BS) {
            const double h = dred[jq + i];
            Hd[i + (int64_t)(jq - 1) * ldh] = h;
            g[i] = h;
            coef[i] = 0.0;
            hs += h * h;
        }
        hs = wave_sum(hs);
        if (lane == 0) rsum[wv] = hs;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int q = 0; q < NW; ++q) t += rsum[q];
            scal[0] = t;
            sv[0] = 0.0;
            sv[1] = 1.0;
            sv[2] = 0.0;
        }
        return;
    }
    // a = Q^T u finishes column jq - 1
    double aa = 0.0, ab = 0.0;
    for (int i = tid; i < jq; i += BS) {
        const double a = dred[i];
        sa[i] = a;
        coef[i] = a;
        aa += a * a;
        ab += a * dred[jq + i];
    }
    aa = wave_sum(aa);
    ab = wave_sum(ab);
    if (lane == 0) {
        rsum[wv] = aa;
        rsum[NW + wv] = ab;
    }
    __syncthreads();
    if (tid == 0) {
        double ta = 0.0;
        for (int q = 0; q < NW; ++q) ta += rsum[q];
        const double uu = dred[2 * jq];
        const double beta = sqrt(fmax(uu - ta, 0.0));
        const double zn = sqrt(scal[0] + uu);
        s_inv = (beta > tol * zn && beta > 0.0) ? 1.0 / beta : 0.0;
        Hd[jq + (int64_t)(jq - 1) * ldh] = beta;
    }
    for (int i = tid; i < jq; i += BS) Hd[i + (int64_t)(jq - 1) * ldh] += sa[i];
    __syncthreads();
    const double inv = s_inv;
    if (kind == DCGS_LAST) {
        if (tid == 0) {
            sv[0] = inv;
            sv[1] = 0.0;
            sv[2] = 0.0;
        }
        return;
    }
    // c = Hbar_jq a ((jq + 1) entries, columns 0..jq-1 final)
    for (int i = tid; i <= jq; i += BS) {
        double t = 0.0;
#pragma unroll 8
        for (int l = 0; l < jq; ++l) t += Hd[i + (int64_t)l * ldh] * sa[l];
        sc[i] = t;
    }
    __syncthreads();
    double tab = 0.0;
    if (tid == 0) {
        for (int q = 0; q < NW; ++q) tab += rsum[NW + q];
    }
    // h of op(q_jq): provisional column jq
    double hs = 0.0;
    for (int i = tid; i < jq; i += BS) {
        const double h = (dred[jq + i] - sc[i]) * inv;
        Hd[i + (int64_t)jq * ldh] = h;
        g[i] = h;   // completed below
        hs += h * h;
    }
    hs = wave_sum(hs);
    __syncthreads();
    if (lane == 0) rsum[wv] = hs;
    __syncthreads();
    if (tid == 0) {
        const double uw = dred[2 * jq + 1];
        const double hj = ((uw - tab) * inv - sc[jq]) * inv;
        Hd[jq + (int64_t)jq * ldh] = hj;
        double t = 0.0;
        for (int q = 0; q < NW; ++q) t += rsum[q];
        scal[0] = t + hj * hj;
        const double gamma = (sc[jq] * inv + hj) * inv;
        sv[0] = inv;
        sv[1] = inv;
        sv[2] = gamma;
        s_gamma = gamma;
    }
    __syncthreads();
    const double gamma = s_gamma;
    for (int i = tid; i < jq; i += BS) g[i] = sc[i] * inv + g[i] - gamma * sa[i];
}

// q_out = (u - Q a) / beta  and  u_out = s_w w - gamma u - Q g  in one pass
// over Q (either output may be null; a null u or w counts as zero).
__global__ __launch_bounds__(BS) void k_dupdate(const double* __restrict__ V, int64_t ldv, int64_t n,
                                                int jq, const double* __restrict__ coef,
                                                const double* __restrict__ u,
                                                const double* __restrict__ w,
                                                double* __restrict__ q_out,
                                                double* __restrict__ u_out) {
    __shared__ double as[CGS_JMAX_ALL + 8], gs[CGS_JMAX_ALL + 8];
    for (int c = threadIdx.x; c < CGS_JMAX_ALL + 8; c += BS) {
        as[c] = c < jq ? coef[c] : 0.0;
        gs[c] = c < jq ? coef[CGS_JMAX_ALL + c] : 0.0;
    }
    const double inv = coef[2 * CGS_JMAX_ALL], sw = coef[2 * CGS_JMAX_ALL + 1],
                 gamma = coef[2 * CGS_JMAX_ALL + 2];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * BS * RPT + threadIdx.x;
    double qa[RPT], ug[RPT], uv[RPT], wv[RPT];
    int64_t rr[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int64_t r = base + (int64_t)i * BS;
        rr[i] = r < n ? r : n - 1;
        uv[i] = u ? u[rr[i]] : 0.0;
        wv[i] = w ? w[rr[i]] : 0.0;
        qa[i] = 0.0;
        ug[i] = 0.0;
    }
    for (int c0 = 0; c0 < jq; c0 += 8) {
        double v[8][RPT];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const double* col = V + (int64_t)min(c0 + c, jq - 1) * ldv;
#pragma unroll
            for (int i = 0; i < RPT; ++i) v[c][i] = col[rr[i]];
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const double ac = as[c0 + c], gc = gs[c0 + c];
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                qa[i] += v[c][i] * ac;
                ug[i] += v[c][i] * gc;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        if (base + (int64_t)i * BS < n) {
            if (q_out) q_out[rr[i]] = (uv[i] - qa[i]) * inv;
            if (u_out) u_out[rr[i]] = sw * wv[i] - gamma * uv[i] - ug[i];
        }
    }
}

// k_dproj and k_dupdate on row pairs (16-byte loads; even n, even ldv and
// 16-byte aligned vectors, as for k_proj2).
__global__ __launch_bounds__(BS) void k_dproj2(const double* __restrict__ V, int64_t ldv, int64_t n,
                                               int jq, const double* __restrict__ u,
                                               const double* __restrict__ w,
                                               double* __restrict__ partial, int nb) {
    constexpr int CH = CT / 2;
    constexpr int RP = RPT / 2;
    __shared__ double red[NW * CT];
    const int64_t base = (int64_t)blockIdx.x * BS * RPT + 2 * threadIdx.x;
    double2 ur[RP], wr[RP];
    int64_t rr[RP];
#pragma unroll
    for (int i = 0; i < RP; ++i) {
        const int64_t r = base + (int64_t)i * 2 * BS;
        rr[i] = r < n ? r : n - 2;
        ur[i] = (u && r < n) ? *reinterpret_cast<const double2*>(u + rr[i]) : make_double2(0.0, 0.0);
        wr[i] = (w && r < n) ? *reinterpret_cast<const double2*>(w + rr[i]) : make_double2(0.0, 0.0);
    }
    {
        double sc[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < RP; ++i) {
            sc[0] += ur[i].x * ur[i].x;
            sc[0] += ur[i].y * ur[i].y;
            sc[1] += ur[i].x * wr[i].x;
            sc[1] += ur[i].y * wr[i].y;
            sc[2] += wr[i].x * wr[i].x;
            sc[2] += wr[i].y * wr[i].y;
        }
        block_reduce_store<3>(sc, 3, red, partial + (int64_t)(2 * jq) * nb + blockIdx.x, nb);
        __syncthreads();
    }
    for (int c0 = 0; c0 < jq; c0 += CH) {
        double acc[2 * CH];
#pragma unroll
        for (int c = 0; c < 2 * CH; ++c) acc[c] = 0.0;
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const double* col = V + (int64_t)min(c0 + c, jq - 1) * ldv;
#pragma unroll
            for (int i = 0; i < RP; ++i) {
                const double2 v = *reinterpret_cast<const double2*>(col + rr[i]);
                acc[c] += v.x * ur[i].x;
                acc[c] += v.y * ur[i].y;
                acc[CH + c] += v.x * wr[i].x;
                acc[CH + c] += v.y * wr[i].y;
            }
        }
        const int cnt = min(CH, jq - c0);
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
        for (int c = 0; c < 2 * CH; ++c) {
            if ((c % CH) < cnt) {
                const double v = wave_sum(acc[c]);
                if (lane == 0) red[wv * CT + c] = v;
            }
        }
        __syncthreads();
        for (int c = threadIdx.x; c < 2 * CH; c += BS) {
            if ((c % CH) >= cnt) continue;
            double t = 0.0;
            for (int q = 0; q < NW; ++q) t += red[q * CT + c];
            const int col = c < CH ? c0 + c : jq + c0 + (c - CH);
            partial[(int64_t)col * nb + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(BS) void k_dupdate2(const double* __restrict__ V, int64_t ldv, int64_t n,
                                                 int jq, const double* __restrict__ coef,
                                                 const double* __restrict__ u,
                                                 const double* __restrict__ w,
                                                 double* __restrict__ q_out,
                                                 double* __restrict__ u_out) {
    constexpr int RP = RPT / 2;
    __shared__ double as[CGS_JMAX_ALL + 8], gs[CGS_JMAX_ALL + 8];
    for (int c = threadIdx.x; c < CGS_JMAX_ALL + 8; c += BS) {
        as[c] = c < jq ? coef[c] : 0.0;
        gs[c] = c < jq ? coef[CGS_JMAX_ALL + c] : 0.0;
    }
    const double inv = coef[2 * CGS_JMAX_ALL], sw = coef[2 * CGS_JMAX_ALL + 1],
                 gamma = coef[2 * CGS_JMAX_ALL + 2];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * BS * RPT + 2 * threadIdx.x;
    double2 qa[RP], ug[RP], uv[RP], wv[RP];
    int64_t rr[RP];
#pragma unroll
    for (int i = 0; i < RP; ++i) {
        const int64_t r = base + (int64_t)i * 2 * BS;
        rr[i] = r < n ? r : n - 2;
        uv[i] = u ? *reinterpret_cast<const double2*>(u + rr[i]) : make_double2(0.0, 0.0);
        wv[i] = w ? *reinterpret_cast<const double2*>(w + rr[i]) : make_double2(0.0, 0.0);
        qa[i] = make_double2(0.0, 0.0);
        ug[i] = make_double2(0.0, 0.0);
    }
    for (int c0 = 0; c0 < jq; c0 += 8) {
        double2 v[8][RP];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const double* col = V + (int64_t)min(c0 + c, jq - 1) * ldv;
#pragma unroll
            for (int i = 0; i < RP; ++i) v[c][i] = *reinterpret_cast<const double2*>(col + rr[i]);
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const double ac = as[c0 + c], gc = gs[c0 + c];
#pragma unroll
            for (int i = 0; i < RP; ++i) {
                qa[i].x += v[c][i].x * ac;
                qa[i].y += v[c][i].y * ac;
                ug[i].x += v[c][i].x * gc;
                ug[i].y += v[c][i].y * gc;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < RP; ++i) {
        if (base + (int64_t)i * 2 * BS < n) {
            if (q_out)
                *reinterpret_cast<double2*>(q_out + rr[i]) =
                    make_double2((uv[i].x - qa[i].x) * inv, (uv[i].y - qa[i].y) * inv);
            if (u_out)
                *reinterpret_cast<double2*>(u_out + rr[i]) =
                    make_double2(sw * wv[i].x - gamma * uv[i].x - ug[i].x,
                                 sw * wv[i].y - gamma * uv[i].y - ug[i].y);
        }
    }
}

}  // namespace

int cgs_blocks(int64_t n) {
    // one block per BS * RPT rows; the partial sums are reduced in a second kernel
    const int64_t nb = (n + BS * RPT - 1) / (BS * RPT);
    PPA_REQUIRE(nb <= (int64_t(1) << 24), "vector too long for the Gram-Schmidt kernels");
    return (int)std::max<int64_t>(1, nb);
}

int ritz_blocks(int64_t n) {
    return (int)std::min<int64_t>(4 * (int64_t)cgs_blocks(n), std::max(cgs_blocks(n), 2048));
}

// blocks of the fused update-projection kernels (one row per thread, or per
// lane pair for the half-row form)
static int cgs_blocks_fused(int64_t n, int rows_per_block) {
    const int64_t nb = (n + rows_per_block - 1) / rows_per_block;
    PPA_REQUIRE(nb <= (int64_t(1) << 27), "vector too long for the Gram-Schmidt kernels");
    return (int)std::max<int64_t>(1, nb);
}

void carve_cgs2(Carver& c, int64_t n, Cgs2Ws& ws) {
    ws.nb = cgs_blocks(n);
    ws.nbf = cgs_blocks_fused(n, BS);
    ws.nbh = cgs_blocks_fused(n, BS / 2);
    ws.partial = c.take<double>(std::max<size_t>((size_t)(2 * CGS_JMAX_ALL + 4) * ws.nb,
                                                 (size_t)CGS_JFUSED * ws.nbh));
    ws.dred = c.take<double>(2 * CGS_JMAX_ALL + 4);
    ws.coef = c.take<double>(2 * CGS_JMAX_ALL + 8);
    ws.h1 = c.take<double>(CGS_JMAX_ALL);
    ws.h2 = c.take<double>(CGS_JMAX_ALL);
    ws.scal = c.take<double>(4);
    ws.t = c.take<double>((size_t)n);
}

static unsigned sgrid(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
}

// the row-pair kernels (16-byte loads) apply for even n, even ldv and
// 16-byte aligned vectors
static bool pairs_ok(int64_t n, int64_t ldv, std::initializer_list<const void*> ptrs) {
    bool ok = n >= 2 && n % 2 == 0 && ldv % 2 == 0;
    for (const void* p : ptrs) ok = ok && reinterpret_cast<uintptr_t>(p) % 16 == 0;
    return ok;
}

static void proj(int64_t n, int j, const double* V, int64_t ldv, const double* w, double* partial,
                 int nb, int with_norm, hipStream_t s) {
    if (pairs_ok(n, ldv, {V, w}))
        hipLaunchKernelGGL(k_proj2, dim3(nb), dim3(BS), 0, s, V, ldv, n, j, w, partial, nb, with_norm);
    else
        hipLaunchKernelGGL(k_proj, dim3(nb), dim3(BS), 0, s, V, ldv, n, j, w, partial, nb, with_norm);
    PPA_HIP(hipGetLastError());
}

static void update(int64_t n, int j, const double* V, int64_t ldv, const double* h, const double* t,
                   double* out, double* partial, int nb, hipStream_t s) {
    if (pairs_ok(n, ldv, {V, t, out}))
        hipLaunchKernelGGL(k_update2, dim3(nb), dim3(BS), 0, s, V, ldv, n, j, h, t, out, partial, nb);
    else
        hipLaunchKernelGGL(k_update, dim3(nb), dim3(BS), 0, s, V, ldv, n, j, h, t, out, partial, nb);
    PPA_HIP(hipGetLastError());
}

static void reduce_cols(const double* partial, int nb, int ncols, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_cols, dim3(ncols), dim3(BS), 0, s, partial, nb, out);
    PPA_HIP(hipGetLastError());
}

void launch_gram(int64_t n, int j, const double* V, int64_t ldv, const double* W, int ncols,
                 double* G_d, Cgs2Ws& ws, hipStream_t s) {
    PPA_REQUIRE(j >= 1 && j <= CGS_JMAX_ALL - 1 && ncols >= 1, "gram: sizes out of range");
    for (int c = 0; c < ncols; ++c) {
        proj(n, j, V, ldv, W + (size_t)c * ldv, ws.partial, ws.nb, 0, s);
        reduce_cols(ws.partial, ws.nb, j, G_d + (size_t)c * j, s);
    }
}

void launch_cgs2(int64_t n, int j, const double* V, int64_t ldv, const double* w, double* w_out,
                 double* Hcol_d, double* v_next, double breakdown_tol, Cgs2Ws& ws,
                 hipStream_t s) {
    PPA_REQUIRE(j >= 1 && j <= CGS_JMAX_ALL - 1, "cgs2: basis size %d out of range", j);
    const int nb = ws.nb;
    // pass 1: h1 = V^T w and ||w_in||^2
    proj(n, j, V, ldv, w, ws.partial, nb, 1, s);
    reduce_cols(ws.partial, nb, j + 1, ws.h1, s);   // h1[0..j-1], h1[j] = ||w_in||^2
    // reorthogonalisation: t = w - V h1, h2 = V^T t (one pass over V when
    // the basis fits the fused kernel's registers)
    if (j <= CGS_JFUSED) {
        const int nbf = j <= 16 ? ws.nbf : ws.nbh;
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(nbf), dim3(BS), 0, s, V, ldv, n, j, ws.h1, w, ws.t,
                               ws.partial, nbf);
        };
        if (j <= 4)
            go(k_update_proj<4>);
        else if (j <= 8)
            go(k_update_proj<8>);
        else if (j <= 16)
            go(k_update_proj<16>);
        else if (j <= 32)
            go(k_update_proj_halves<16>);
        else
            go(k_update_proj_halves<32>);
        PPA_HIP(hipGetLastError());
        reduce_cols(ws.partial, nbf, j, ws.h2, s);
    } else {
        update(n, j, V, ldv, ws.h1, w, ws.t, nullptr, nb, s);
        proj(n, j, V, ldv, ws.t, ws.partial, nb, 0, s);
        reduce_cols(ws.partial, nb, j, ws.h2, s);
    }
    // w_out = t - V h2 and ||w_out||^2
    update(n, j, V, ldv, ws.h2, ws.t, w_out, ws.partial, nb, s);
    if (v_next) {
        // reduction, Hessenberg column and v_next = w_out / beta in one launch
        // at most 1024 blocks: each repeats the norm's reduction, then scales
        // its grid-stride share of w_out
        hipLaunchKernelGGL(k_finalize_scale, dim3(std::min(sgrid(n), 1024u)), dim3(BS), 0, s, ws.partial, nb, ws.h1,
                           ws.h2, j, ws.scal, Hcol_d, breakdown_tol, w_out, v_next, n);
        PPA_HIP(hipGetLastError());
        return;
    }
    reduce_cols(ws.partial, nb, 1, ws.scal + 1, s);
    hipLaunchKernelGGL(k_cgs_finalize, dim3(1), dim3(256), 0, s, ws.h1, ws.h2, j, ws.scal, Hcol_d,
                       breakdown_tol);
    PPA_HIP(hipGetLastError());
}

void launch_dcgs_step(int kind, int64_t n, int jq, const double* V, int64_t ldv, const double* u,
                      const double* w, double* Hd, int64_t ldh, double* q_out, double* u_out,
                      double breakdown_tol, Cgs2Ws& ws, hipStream_t s) {
    PPA_REQUIRE(jq >= 1 && jq <= CGS_JMAX_ALL - 1, "delayed Gram-Schmidt: basis size %d out of range", jq);
    PPA_REQUIRE((kind == DCGS_FIRST && w && !u) || (kind == DCGS_LAGGED && u && w) ||
                    (kind == DCGS_LAST && u && !w),
                "delayed Gram-Schmidt: operands do not match the step kind");
    const int nb = ws.nb;
    const bool pairs = pairs_ok(n, ldv, {V, u, w, q_out, u_out});
    if (pairs)
        hipLaunchKernelGGL(k_dproj2, dim3(nb), dim3(BS), 0, s, V, ldv, n, jq, u, w, ws.partial, nb);
    else
        hipLaunchKernelGGL(k_dproj, dim3(nb), dim3(BS), 0, s, V, ldv, n, jq, u, w, ws.partial, nb);
    PPA_HIP(hipGetLastError());
    reduce_cols(ws.partial, nb, 2 * jq + 3, ws.dred, s);
    hipLaunchKernelGGL(k_dcoef, dim3(1), dim3(BS), 0, s, kind, jq, ws.dred, Hd, ldh, ws.coef, ws.scal,
                       breakdown_tol);
    PPA_HIP(hipGetLastError());
    if (pairs)
        hipLaunchKernelGGL(k_dupdate2, dim3(nb), dim3(BS), 0, s, V, ldv, n, jq, ws.coef, u, w,
                           kind == DCGS_FIRST ? nullptr : q_out, kind == DCGS_LAST ? nullptr : u_out);
    else
        hipLaunchKernelGGL(k_dupdate, dim3(nb), dim3(BS), 0, s, V, ldv, n, jq, ws.coef, u, w,
                           kind == DCGS_FIRST ? nullptr : q_out, kind == DCGS_LAST ? nullptr : u_out);
    PPA_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- MFMA GEMM
// C[:, 0:kout] = V[:, 0:kin] Q, FP64 on v_mfma_f64_16x16x4f64.
// Block = 4 waves; each wave owns RT tiles of 16 rows and all NT tiles of 16
// output columns.  Q (zero-padded to KP x 16*NT) is staged in LDS once.
// Operand layout of the 16x16x4 FP64 MFMA (wave of 64 lanes):
//   A[i][k] in lane i + 16k;  B[k][j] in lane j + 16k;
//   D[i][j] in lane j + 16 (i % 4), element i / 4.
// The product is formed transposed, C_tile^T = Q_tile^T V_tile^T (A from Q,
// B from V), so that each lane's outputs lie in one row of C and a store
// instruction covers 16 consecutive rows.
typedef double v4d __attribute__((ext_vector_type(4)));


template <int NT, int RT>
__global__ __launch_bounds__(256) void k_gemm_tall(int64_t n, int kin, int kout,
                                                   const double* __restrict__ V, int64_t ldv,
                                                   const double* __restrict__ Q,
                                                   double* __restrict__ C, int64_t ldc) {
    extern __shared__ double Qs[];
    constexpr int NP = NT * 16;
    const int KP = (kin + 3) & ~3;
    for (int idx = threadIdx.x; idx < KP * NP; idx += 256) {
        const int kk = idx / NP, cc = idx % NP;
        Qs[idx] = (kk < kin && cc < kout) ? Q[(int64_t)cc * kin + kk] : 0.0;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    // the block stages Q once and walks row chunks of 4 waves x 16 RT rows
    for (int64_t chunk = blockIdx.x; chunk * 4 * 16 * RT < n; chunk += gridDim.x) {
    const int64_t rbase = (chunk * 4 + wave) * (16 * RT);
    v4d acc[RT][NT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[rt][t] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < KP; k0 += 4) {
        const int kc = k0 + lk;
        double a[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int64_t row = rbase + rt * 16 + li;
            a[rt] = (row < n && kc < kin) ? V[(int64_t)kc * ldv + row] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const double bq = Qs[kc * NP + t * 16 + li];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
                acc[rt][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(bq, a[rt], acc[rt][t], 0, 0, 0);
        }
    }
    // D = Q_tile^T V_tile^T: lane li + 16 lk holds rows li of columns
    // t*16 + 4e + lk, so a store writes 16 consecutive rows of 4 columns
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int64_t row = rbase + rt * 16 + li;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int col = t * 16 + 4 * e + lk;
                if (row < n && col < kout) C[(int64_t)col * ldc + row] = acc[rt][t][e];
            }
        }
    }
}

void launch_gemm_tall(int64_t n, int kin, int kout, const double* V, int64_t ldv, const double* Q_d,
                      double* C, int64_t ldc, hipStream_t s) {
    PPA_REQUIRE(kin >= 1 && kin <= 128 && kout >= 1 && kout <= 64, "gemm: kin %d / kout %d out of range",
                kin, kout);
    if (n <= 0) return;
    constexpr int RT = 2;
    // enough blocks to fill the chip several times over; each stages Q once
    const unsigned grid = (unsigned)std::min<int64_t>((n + 4 * 16 * RT - 1) / (4 * 16 * RT), 2048);
    const int KP = (kin + 3) & ~3;
    const int NT = (kout + 15) / 16;
    const size_t lds = (size_t)KP * NT * 16 * sizeof(double);
    switch (NT) {
        case 1: hipLaunchKernelGGL((k_gemm_tall<1, RT>), dim3(grid), dim3(256), lds, s, n, kin, kout, V, ldv, Q_d, C, ldc); break;
        case 2: hipLaunchKernelGGL((k_gemm_tall<2, RT>), dim3(grid), dim3(256), lds, s, n, kin, kout, V, ldv, Q_d, C, ldc); break;
        case 3: hipLaunchKernelGGL((k_gemm_tall<3, RT>), dim3(grid), dim3(256), lds, s, n, kin, kout, V, ldv, Q_d, C, ldc); break;
        default: hipLaunchKernelGGL((k_gemm_tall<4, RT>), dim3(grid), dim3(256), lds, s, n, kin, kout, V, ldv, Q_d, C, ldc); break;
    }
    PPA_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- dots
namespace {
__global__ __launch_bounds__(BS) void k_dots(int64_t n, DotList L, double* __restrict__ partial,
                                             int nb) {
    __shared__ double red[NW * 8];
    const RowRange rr = rows_of_block(n, nb);
    for (int g = 0; g < L.count; g += 8) {
        double acc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = 0.0;
        const int cnt = min(8, L.count - g);
        for (int64_t r = rr.beg + threadIdx.x; r < rr.end; r += BS) {
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c < cnt) acc[c] += L.a[g + c][r] * L.b[g + c][r];
        }
        block_reduce_store<8>(acc, cnt, red, partial + (int64_t)g * nb + blockIdx.x, nb);
        __syncthreads();
    }
}

__global__ __launch_bounds__(BS) void k_combo_norms(int64_t n, ComboList L,
                                                    double* __restrict__ partial, int nb) {
    __shared__ double red[NW * 8];
    const RowRange rr = rows_of_block(n, nb);
    for (int g = 0; g < L.count; g += 8) {
        double acc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = 0.0;
        const int cnt = min(8, L.count - g);
        for (int64_t r = rr.beg + threadIdx.x; r < rr.end; r += BS) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                if (c < cnt) {
                    double v = 0.0;
#pragma unroll
                    for (int t = 0; t < 3; ++t)
                        if (L.v[g + c][t]) v += L.c[g + c][t] * L.v[g + c][t][r];
                    acc[c] += v * v;
                }
            }
        }
        block_reduce_store<8>(acc, cnt, red, partial + (int64_t)g * nb + blockIdx.x, nb);
        __syncthreads();
    }
}

__global__ void k_copy_complex(int64_t n, const double* __restrict__ Y, int64_t ldy,
                               const int* __restrict__ cre, const int* __restrict__ cim,
                               const double* __restrict__ scale, int ncols, double* __restrict__ X) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int c = 0; c < ncols; ++c) {
            const double sr = scale[2 * c], si = scale[2 * c + 1];
            const double re = cre[c] >= 0 ? Y[(int64_t)cre[c] * ldy + i] : 0.0;
            const double im = cim[c] >= 0 ? Y[(int64_t)cim[c] * ldy + i] : 0.0;
            X[2 * ((int64_t)c * n + i)] = sr * re;
            X[2 * ((int64_t)c * n + i) + 1] = si * im;
        }
    }
}

__global__ void k_zero(double* p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}
}  // namespace

void launch_dots(int64_t n, const DotList& L, double* partial, int nb, double* out_d,
                 hipStream_t s) {
    PPA_REQUIRE(L.count >= 1 && L.count <= MAX_DOTS, "dots: bad count");
    hipLaunchKernelGGL(k_dots, dim3(nb), dim3(BS), 0, s, n, L, partial, nb);
    PPA_HIP(hipGetLastError());
    reduce_cols(partial, nb, L.count, out_d, s);
}

void launch_combo_norms(int64_t n, const ComboList& L, double* partial, int nb, double* out_d,
                        hipStream_t s) {
    PPA_REQUIRE(L.count >= 1 && L.count <= MAX_COMBOS, "combo norms: bad count");
    hipLaunchKernelGGL(k_combo_norms, dim3(nb), dim3(BS), 0, s, n, L, partial, nb);
    PPA_HIP(hipGetLastError());
    reduce_cols(partial, nb, L.count, out_d, s);
}

void launch_copy_cols_complex(int64_t n, const double* Y, int64_t ldy, const int* cre,
                              const int* cim, const double* scale, int ncols, double* X,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_copy_complex, dim3(sgrid(n)), dim3(256), 0, s, n, Y, ldy, cre, cim, scale,
                       ncols, X);
    PPA_HIP(hipGetLastError());
}

void launch_zero(double* p, int64_t count, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_zero, dim3(sgrid(count)), dim3(256), 0, s, p, count);
    PPA_HIP(hipGetLastError());
}

}  // namespace ppa
