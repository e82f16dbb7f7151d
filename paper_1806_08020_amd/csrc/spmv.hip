// Fused CSR SpMV + axpy kernels: one coalesced HBM pass per factor of pi(A).
//
// A factor (I - A/theta) of eq. (2.1), or either half of a conjugate-pair
// step, is the same fused operation
//     out = alpha x + beta (A u) + gamma z + delta z2,
// so each degree step streams the CSR arrays once, gathers u, streams x (and
// z, z2 for the double-polynomial epilogue of section 8) and writes out.
//
// Layout and mapping (gfx950):
//  * rows are cut into row blocks of at most SPMV_CHUNK nonzeros; a block of
//    SPMV_BS threads first loads its contiguous nonzero range (colind, values)
//    with unit-stride, non-temporal loads, multiplies by the gathered u and
//    stages the products in LDS, then each thread sums whole rows from LDS and
//    applies the axpy epilogue -- every global access but the gather of u is
//    coalesced;
//  * a row with more than SPMV_CHUNK nonzeros gets a block of its own that
//    reduces it across the block;
//  * block ids are remapped so that each of the 8 XCDs walks one contiguous
//    range of rows: neighbouring row blocks share gathered u lines in the same
//    XCD's L2;
//  * the row sum is accumulated in the value precision (FP64, or FP32 for the
//    FP32 / mixed path), in column order, so results are deterministic.
#include "ppa_internal.hpp"

#include <algorithm>
#include <cmath>

namespace ppa {

__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb / NUM_XCD, r = nb % NUM_XCD;
    const int x = b % NUM_XCD, i = b / NUM_XCD;
    return x * q + min(x, r) + i;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename VT, typename IT, typename OT>
__global__ __launch_bounds__(SPMV_BS) void k_fused_spmv(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
    const VT* __restrict__ val, const int32_t* __restrict__ blk, int nblk,
    const IT* __restrict__ x, const IT* __restrict__ u, const IT* __restrict__ z,
    const IT* __restrict__ z2, OT* __restrict__ out, VT alpha, VT beta, VT gamma, VT delta) {
    __shared__ VT prod[SPMV_CHUNK];
    __shared__ VT red[SPMV_BS / 64];
    const int b = xcd_remap(blockIdx.x, nblk);
    const int r0 = blk[b], r1 = blk[b + 1];
    const int p0 = rowptr[r0], p1 = rowptr[r1];
    const int cnt = p1 - p0;
    const int tid = threadIdx.x;
    if (cnt <= SPMV_CHUNK) {
        constexpr int PER = SPMV_CHUNK / SPMV_BS;
        int32_t c[PER];
        VT v[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = tid + k * SPMV_BS;
            if (i < cnt) {
                c[k] = __builtin_nontemporal_load(colind + p0 + i);
                v[k] = __builtin_nontemporal_load(val + p0 + i);
            }
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = tid + k * SPMV_BS;
            if (i < cnt) prod[i] = v[k] * (VT)u[c[k]];
        }
        __syncthreads();
        for (int r = r0 + tid; r < r1; r += SPMV_BS) {
            const int a = rowptr[r] - p0, e = rowptr[r + 1] - p0;
            VT s = 0;
            for (int q = a; q < e; ++q) s += prod[q];
            VT o = beta * s;
            if (x) o += alpha * (VT)x[r];
            if (z) o += gamma * (VT)z[r];
            if (z2) o += delta * (VT)z2[r];
            out[r] = (OT)o;
        }
    } else {
        // one long row: r1 == r0 + 1
        VT s = 0;
        for (int i = p0 + tid; i < p1; i += SPMV_BS) s += val[i] * (VT)u[colind[i]];
        s = wave_sum(s);
        if ((tid & 63) == 0) red[tid >> 6] = s;
        __syncthreads();
        if (tid == 0) {
            VT t = 0;
            for (int w = 0; w < SPMV_BS / 64; ++w) t += red[w];
            VT o = beta * t;
            if (x) o += alpha * (VT)x[r0];
            if (z) o += gamma * (VT)z[r0];
            if (z2) o += delta * (VT)z2[r0];
            out[r0] = (OT)o;
        }
    }
}

template <typename VT, typename IT, typename OT>
static void run_fused(const Matrix& A, const VT* val, double alpha, const void* x, double beta,
                      const void* u, double gamma, const void* z, double delta, const void* z2,
                      void* o, hipStream_t s) {
    if (A.nblocks == 0) return;
    hipLaunchKernelGGL((k_fused_spmv<VT, IT, OT>), dim3((unsigned)A.nblocks), dim3(SPMV_BS), 0,
                       s, A.rowptr, A.colind, val, A.blk, (int)A.nblocks, (const IT*)x,
                       (const IT*)u, (const IT*)z, (const IT*)z2, (OT*)o, (VT)alpha, (VT)beta,
                       (VT)gamma, (VT)delta);
    PPA_HIP(hipGetLastError());
}

void launch_fused_spmv(const Matrix& A, VecT in, VecT out, double alpha, const void* x,
                       double beta, const void* u, double gamma, const void* z, double delta,
                       const void* z2, void* o, hipStream_t s) {
    PPA_REQUIRE(u != nullptr && o != nullptr, "fused spmv: u and out are required");
    PPA_REQUIRE(o != u, "fused spmv: out must not alias u");
    if (in == VecT::F64 && out == VecT::F64) {
        run_fused<double, double, double>(A, A.v64, alpha, x, beta, u, gamma, z, delta, z2, o, s);
        return;
    }
    PPA_REQUIRE(A.v32 != nullptr, "FP32 path needs FP32 matrix values (want_f32 at create)");
    if (in == VecT::F32 && out == VecT::F32)
        run_fused<float, float, float>(A, A.v32, alpha, x, beta, u, gamma, z, delta, z2, o, s);
    else if (in == VecT::F64 && out == VecT::F32)
        run_fused<float, double, float>(A, A.v32, alpha, x, beta, u, gamma, z, delta, z2, o, s);
    else if (in == VecT::F32 && out == VecT::F64)
        run_fused<float, float, double>(A, A.v32, alpha, x, beta, u, gamma, z, delta, z2, o, s);
    else
        run_fused<float, double, double>(A, A.v32, alpha, x, beta, u, gamma, z, delta, z2, o, s);
}

// ---------------------------------------------------------------- setup
// Per-row structural check (indices in range, strictly increasing) and the
// absolute row sum; one result per block: bad-row count and max row sum.
__global__ __launch_bounds__(256) void k_validate(const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ colind,
                                                  const double* __restrict__ val, int64_t n,
                                                  int* __restrict__ bad,
                                                  double* __restrict__ rmax) {
    __shared__ double smax[256];
    __shared__ int sbad[256];
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double rs = 0.0;
    int nb = 0;
    if (r < n) {
        const int a = rowptr[r], e = rowptr[r + 1];
        if (e < a) nb = 1;
        int prev = -1;
        for (int q = a; q < e; ++q) {
            const int c = colind[q];
            if (c < 0 || c >= n || c <= prev) nb = 1;
            prev = c;
            const double v = val[q];
            if (!(v == v) || fabs(v) == INFINITY) nb = 1;
            rs += fabs(v);
        }
    }
    smax[threadIdx.x] = rs;
    sbad[threadIdx.x] = nb;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
            sbad[threadIdx.x] += sbad[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        bad[blockIdx.x] = sbad[0];
        rmax[blockIdx.x] = smax[0];
    }
}

__global__ void k_cast_f64_f32(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}
__global__ void k_cast_f32_f64(const float* __restrict__ in, double* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (double)in[i];
}

static unsigned stream_grid(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
}

void launch_cast_f64_f32(const double* in, float* out, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_cast_f64_f32, dim3(stream_grid(n)), dim3(256), 0, s, in, out, n);
    PPA_HIP(hipGetLastError());
}
void launch_cast_f32_f64(const float* in, double* out, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_cast_f32_f64, dim3(stream_grid(n)), dim3(256), 0, s, in, out, n);
    PPA_HIP(hipGetLastError());
}

void matrix_setup(Matrix& A, hipStream_t s) {
    const int64_t n = A.n;
    std::vector<int32_t> rp(n + 1);
    PPA_HIP(hipMemcpyAsync(rp.data(), A.rowptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PPA_HIP(hipStreamSynchronize(s));
    PPA_REQUIRE(rp[0] == 0, "rowptr[0] must be 0");
    for (int64_t i = 0; i < n; ++i)
        PPA_REQUIRE(rp[i + 1] >= rp[i], "rowptr must be nondecreasing (row %lld)", (long long)i);
    A.nnz = rp[n];
    // validation + ||A||_inf on the device
    const int64_t nb = (n + 255) / 256;
    int* bad = nullptr;
    double* rmax = nullptr;
    PPA_HIP(hipMalloc(&bad, nb * sizeof(int)));
    PPA_HIP(hipMalloc(&rmax, nb * sizeof(double)));
    hipLaunchKernelGGL(k_validate, dim3((unsigned)nb), dim3(256), 0, s, A.rowptr, A.colind, A.v64,
                       n, bad, rmax);
    PPA_HIP(hipGetLastError());
    std::vector<int> hb(nb);
    std::vector<double> hm(nb);
    PPA_HIP(hipMemcpyAsync(hb.data(), bad, nb * sizeof(int), hipMemcpyDeviceToHost, s));
    PPA_HIP(hipMemcpyAsync(hm.data(), rmax, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    PPA_HIP(hipStreamSynchronize(s));
    PPA_HIP(hipFree(bad));
    PPA_HIP(hipFree(rmax));
    int64_t nbad = 0;
    double nrm = 0.0;
    for (int64_t i = 0; i < nb; ++i) {
        nbad += hb[i];
        nrm = std::max(nrm, hm[i]);
    }
    PPA_REQUIRE(nbad == 0,
                "malformed CSR: %lld rows with out-of-range, unsorted or repeated column "
                "indices or non-finite values",
                (long long)nbad);
    A.norm_inf = nrm;
    // greedy row-block partition
    std::vector<int32_t> blk;
    blk.reserve(n / 64 + 2);
    blk.push_back(0);
    int64_t r = 0;
    while (r < n) {
        const int64_t start = r, base = rp[r];
        if (rp[r + 1] - base > SPMV_CHUNK) {
            ++r;
        } else {
            while (r < n && rp[r + 1] - base <= SPMV_CHUNK && r - start < SPMV_MAXROWS) ++r;
        }
        blk.push_back((int32_t)r);
    }
    A.nblocks = (int64_t)blk.size() - 1;
    PPA_HIP(hipMalloc(&A.blk, blk.size() * sizeof(int32_t)));
    PPA_HIP(hipMemcpyAsync(A.blk, blk.data(), blk.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    PPA_HIP(hipStreamSynchronize(s));
}

}  // namespace ppa
