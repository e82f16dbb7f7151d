// Internal declarations of libppa (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ppa.h"

namespace ppa {

using cplx = std::complex<double>;

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(int code, const char* fmt, ...);
void hip_check(hipError_t e, const char* what, const char* file, int line);
#define PPA_HIP(x) ::ppa::hip_check((x), #x, __FILE__, __LINE__)
#define PPA_REQUIRE(cond, ...) \
    do { if (!(cond)) ::ppa::fail(PPA_ERR_INVALID, __VA_ARGS__); } while (0)

// ---------------------------------------------------------------- handles
// SpMV row-block partition: each block holds at most SPMV_CHUNK nonzeros and
// at most SPMV_MAXROWS rows, or exactly one row longer than SPMV_CHUNK.
#ifndef PPA_SPMV_BS
#define PPA_SPMV_BS 256
#endif
#ifndef PPA_SPMV_CHUNK
#define PPA_SPMV_CHUNK 2048
#endif
constexpr int SPMV_BS = PPA_SPMV_BS;
constexpr int SPMV_CHUNK = PPA_SPMV_CHUNK;
// the plain kernel's second block shape: 64 threads, 256 nonzeros
#ifndef PPA_SPMV_BS_S
#define PPA_SPMV_BS_S 64
#endif
#ifndef PPA_SPMV_CHUNK_S
#define PPA_SPMV_CHUNK_S 256
#endif
constexpr int SPMV_BS_S = PPA_SPMV_BS_S;
constexpr int SPMV_CHUNK_S = PPA_SPMV_CHUNK_S;
constexpr int SPMV_MAXROWS = PPA_SPMV_CHUNK;
// MI355X: 8 accelerator complex dies, workgroups dispatched round-robin.
constexpr int NUM_XCD = 8;

// Windowed SpMV (matrices whose row blocks touch a narrow column range, e.g.
// band matrices with scattered columns): a block stages u[cmin .. cmax] of its
// rows in LDS and gathers from there.
#ifndef PPA_SPMV_WBS
#define PPA_SPMV_WBS 1024
#endif
#ifndef PPA_SPMV_WCHUNK_F32
#define PPA_SPMV_WCHUNK_F32 8192
#endif
constexpr int SPMV_WBS = PPA_SPMV_WBS;                // threads per windowed block
constexpr int SPMV_WCHUNK_F32 = PPA_SPMV_WCHUNK_F32;  // nonzeros per windowed block, FP32 values
#ifndef PPA_SPMV_WCHUNK_F64
#define PPA_SPMV_WCHUNK_F64 8192
#endif
#ifndef PPA_SPMV_WIN_LDS_MAX
#define PPA_SPMV_WIN_LDS_MAX (160 * 1024)
#endif
constexpr int SPMV_WCHUNK_F64 = PPA_SPMV_WCHUNK_F64;  // nonzeros per windowed block, FP64 values
constexpr int SPMV_WIN_LDS_MAX = PPA_SPMV_WIN_LDS_MAX;   // LDS budget of one windowed block

struct Window {
    bool on = false;                 // selected for this value type
    int4* bm = nullptr;              // device, per block {r0, r1, p0, p1}, {cmin, span, 0, 0}
    int align = 1;                   // block ranges start at multiples of this
    int64_t nblocks = 0;
    int span_max = 0;
    size_t lds_bytes = 0;
};

// Sliding-window SpMV (band matrices): one persistent block per CU walks a
// segment of consecutive row chunks and keeps u in an LDS ring of
// SPMV_RING_F64 / SPMV_RING_F32 entries; each chunk only adds the columns
// it reaches beyond the previous ones.  LDS per block: the ring and two
// product buffers of one chunk, 160 KB in both precisions.
#ifndef PPA_SPMV_RING_F64
#define PPA_SPMV_RING_F64 12288
#endif
#ifndef PPA_SPMV_RING_F32
#define PPA_SPMV_RING_F32 24576
#endif
#ifndef PPA_SPMV_RCHUNK_F64
#define PPA_SPMV_RCHUNK_F64 4096
#endif
#ifndef PPA_SPMV_RCHUNK_F32
#define PPA_SPMV_RCHUNK_F32 8192
#endif
#ifndef PPA_SPMV_RBS_F64
#define PPA_SPMV_RBS_F64 1024
#endif
#ifndef PPA_SPMV_RBS_F32
#define PPA_SPMV_RBS_F32 1024
#endif
#ifndef PPA_SPMV_RPERCU_F64
#define PPA_SPMV_RPERCU_F64 1
#endif
#ifndef PPA_SPMV_RPERCU_F32
#define PPA_SPMV_RPERCU_F32 1
#endif
#ifndef PPA_SPMV_RING_NEW
#define PPA_SPMV_RING_NEW 1
#endif
#ifndef PPA_SPMV_RING_D
#define PPA_SPMV_RING_D 3
#endif
constexpr int SPMV_RING_F64 = PPA_SPMV_RING_F64;      // ring entries, FP64 values (96 KB)
constexpr int SPMV_RING_F32 = PPA_SPMV_RING_F32;      // ring entries, FP32 values (96 KB)
constexpr int SPMV_RCHUNK_F64 = PPA_SPMV_RCHUNK_F64;  // nonzeros per chunk, FP64 values
constexpr int SPMV_RCHUNK_F32 = PPA_SPMV_RCHUNK_F32;  // nonzeros per chunk, FP32 values
constexpr int SPMV_RBS_F64 = PPA_SPMV_RBS_F64;        // threads per block, FP64 values
constexpr int SPMV_RBS_F32 = PPA_SPMV_RBS_F32;        // threads per block, FP32 values
constexpr int SPMV_RPERCU_F64 = PPA_SPMV_RPERCU_F64;  // blocks (segments) per CU, FP64 values
constexpr int SPMV_RPERCU_F32 = PPA_SPMV_RPERCU_F32;  // blocks (segments) per CU, FP32 values
constexpr int SPMV_RING_NEW = PPA_SPMV_RING_NEW;      // new ring columns per thread and chunk
constexpr int SPMV_RING_D = PPA_SPMV_RING_D;          // chunks held in registers

// Two factors of the polynomial per pass, for matrices of small bandwidth
// h (every entry has |column - row| <= h).  Block b (SPMV_TWO_BS threads,
// one per CU) owns output rows [r0, r1); it stages u on [w0, w1) =
// [r0 - 2h, r1 + 2h) in LDS, computes the first factor on rows [e0, e1) =
// [r0 - h, r1 + h) into LDS and the second factor on its own rows from
// there (all ranges clipped to [0, n)).  Per block three records
// {r0, r1, e0, e1}, {w0, w1, c0, c1}, {c2, 0, 0, 0}: sub-chunks [c0, c1)
// cover rows [e0, e1) and [c1, c2) rows [r0, r1), each sub-chunk
// {row begin, row end, nonzero begin, nonzero end} of whole rows with at
// most SPMV_TWO_CH nonzeros.
#ifndef PPA_SPMV_TWO_CH
#define PPA_SPMV_TWO_CH 4096
#endif
constexpr int SPMV_TWO_BS = 1024;
constexpr int SPMV_TWO_CH = PPA_SPMV_TWO_CH;

struct TwoStep {
    bool on64 = false, on32 = false;   // in use for this value type
    bool ok64 = false, ok32 = false;   // fits the LDS for this value type
    int4* blk = nullptr;               // device, three records per block
    int4* sub = nullptr;               // device, sub-chunk records
    int64_t nblk = 0, nsub = 0;
    int h = 0, wmax = 0, emax = 0;
};

struct Ring {
    bool on = false;
    int4* rm = nullptr;              // device, per chunk {r0, r1, p0, p1}, {lo, hi, 0, 0}
    int4* seg = nullptr;             // device, per segment {t0, t1, 0, 0}
    int align = 1;
    int64_t nchunks = 0, nseg = 0;
    size_t lds_bytes = 0;
};

// Column-run windows of the plain kernel's large blocks.  The columns a block
// gathers form a few contiguous runs for stencil and band matrices (a 3-D
// 7-point stencil: the planes below and above and the rows around it).  Per
// block the setup stores the runs (sorted, disjoint, starts rounded down and
// ends up to multiples of 4 entries, gaps of at most SPMV_RUNS_GAP entries
// bridged) as 16 ints:
//   [0] number of runs (0: the block gathers from global memory)
//   [1] LDS entries of all runs
//   [2 + k] first column of run k (k < SPMV_RUNS_MAX; unused: INT32_MAX)
//   [2 + SPMV_RUNS_MAX + k - 1] LDS offset of run k, k >= 1 (unused: INT32_MAX)
// The runs also cover the block's own rows.  The block copies its runs of u
// into LDS with 16-byte loads issued together with its matrix stream (they do
// not wait for the column indices), then reads every gathered entry from LDS,
// and x[r] too when x is u.  A block whose runs exceed
// SPMV_RUNS_LDS bytes in the value type gathers from global memory.
#ifndef PPA_SPMV_RUNS_MAX
#define PPA_SPMV_RUNS_MAX 7
#endif
#ifndef PPA_SPMV_RUNS_LDS
#define PPA_SPMV_RUNS_LDS 10240
#endif
#ifndef PPA_SPMV_RUNS_GAP
#define PPA_SPMV_RUNS_GAP 16
#endif
constexpr int SPMV_RUNS_MAX = PPA_SPMV_RUNS_MAX;
constexpr int SPMV_RUNS_LDS = PPA_SPMV_RUNS_LDS;
constexpr int SPMV_RUNS_GAP = PPA_SPMV_RUNS_GAP;
constexpr int SPMV_RUNS_REC = 16;
static_assert(2 + 2 * SPMV_RUNS_MAX - 1 <= SPMV_RUNS_REC, "run record holds 16 ints");

struct Runs {
    int32_t* rec = nullptr;          // device, SPMV_RUNS_REC ints per large block
    int64_t nblocks = 0;
    int64_t nwin64 = 0, nwin32 = 0;  // blocks whose runs fit the LDS budget per value type
    bool on64 = false, on32 = false; // the plain large-block kernel uses them
};

// The windowed and sliding-window variants are timed at matrix creation only
// when the plain kernel's tuned pass runs below this rate (GB/s; half the
// MI355X HBM peak).
constexpr double SPMV_STAGED_GATE_GBS = 4000.0;

// Cache policies of the plain SpMV kernel (values match ppa.h's PPA_CACHE_*).
enum { CP_STREAM = 0, CP_KEEP = 1, CP_KEEP_NTST = 2 };

struct Matrix {
    int64_t n = 0, nnz = 0;
    const int32_t* rowptr = nullptr;
    const int32_t* colind = nullptr;
    const double* v64 = nullptr;
    const float* v32 = nullptr;
    float* v32_owned = nullptr;
    int4* bm = nullptr;              // device, per block {r0, r1, p0, p1}
    int64_t nblocks = 0;
    int align = 1;                   // block ranges start at multiples of this (1 or 4)
    int cp64 = CP_KEEP, cp32 = CP_KEEP;   // cache policy of the plain SpMV kernel per value type
    int4* bm_s = nullptr;            // partition into SPMV_CHUNK_S-nonzero blocks
    int64_t nblocks_s = 0;
    int blk64 = 0, blk32 = 0;        // plain kernel block shape per value type: 0 large, 1 small
    bool long_s = false;             // a row needs a block of its own in the small partition
    double norm_inf = 0.0;
    int device = 0;
    Window win64, win32;
    Ring ring64, ring32;
    Runs runs;
    TwoStep two;
    std::vector<int32_t> rp_host;    // host copy of rowptr (setup only)
};

struct Poly {
    std::vector<cplx> roots;    // pi (single) or pi_2 (double), application order
    std::vector<cplx> roots1;   // pi_1 (double polynomial), empty otherwise
    double shift = 0.0;         // the polynomial acts on A - shift I
    bool is_double() const { return !roots1.empty(); }
    int degree() const { return (int)roots.size(); }
    int total_degree() const {
        return is_double() ? (int)(roots.size() * roots1.size()) : (int)roots.size();
    }
};

// ---------------------------------------------------------------- workspace
// Carves 256-byte aligned sub-buffers out of one caller allocation.  With
// base == nullptr it only measures (used by the *_workspace_bytes queries).
struct Carver {
    char* base;
    size_t cap;
    size_t off = 0;
    Carver(void* b, size_t c) : base((char*)b), cap(c) {}
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    void check() const {
        if (base && off > cap)
            fail(PPA_ERR_WORKSPACE, "workspace too small: need %zu bytes, got %zu", off, cap);
    }
    size_t bytes() const { return (off + 255) & ~size_t(255); }
};

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Leading dimension of a block of n-vectors (256-byte aligned columns).
inline int64_t col_ld(int64_t n) { return round_up(n, 32); }

// ---------------------------------------------------------------- kernels
enum class VecT { F64, F32 };

// out = alpha x + beta (A u) + gamma z + delta z2   (x, z, z2 may be null).
// Returns the pass's algorithmic bytes: CSR arrays once (values, int32 column
// indices, int32 row pointers), each distinct input vector once, the output once.
size_t fused_spmv_bytes(const Matrix& A, VecT in, VecT out, const void* x, const void* u,
                        const void* z, const void* z2);
// AY = A Y for the ncols columns of the column-major FP64 block Y (leading
// dimension ld, shared by AY); each column equals the single-column FP64
// pass out = A y bit for bit.  Rows that need a block of their own in the
// small partition send the whole call to the single-column kernel.
void launch_spmm_cols(const Matrix& A, const double* Y, int64_t ld, int ncols, double* AY,
                      hipStream_t s);
size_t launch_fused_spmv(const Matrix& A, VecT in, VecT out, double alpha, const void* x,
                       double beta, const void* u, double gamma, const void* z, double delta,
                       const void* z2, void* o, hipStream_t s);
// Two consecutive factor passes of a chain in one launch (TwoStep): with s
// the first pass's output,
//   s   = a1 u + b1 A u
//   out = a2 x2 + b2 A s + g2 s,   x2 = s (x2s) or u
// where the g2 term is present only with zs.  Each value is bitwise the one
// the two single passes give (same products, same row sums).  Needs
// two_step_on(A, t); u and out in the value type t.  Returns the two
// passes' algorithmic bytes.
bool two_step_on(const Matrix& A, VecT t);
size_t launch_two_step(const Matrix& A, VecT t, double a1, double b1, double a2, double b2, double g2,
                       bool zs, bool x2s, const void* u, void* out, hipStream_t s);
// Records for two factors per pass when the bandwidth lets a block's LDS
// hold its ranges; call during creation (needs rp_host).
void build_two_step(Matrix& A, hipStream_t s);
void matrix_setup(Matrix& A, hipStream_t s);   // validate, norm, partition
// Choose between the plain and the windowed SpMV for each available value
// type: mode 0 times both on a scratch vector (large matrices only), mode 1
// forces the windowed kernel whenever it fits, mode -1 keeps the plain one.
void matrix_tune(Matrix& A, int mode, bool timing, hipStream_t s);
void matrix_release(Matrix& A);
// out = a x + b y + c z (y, z may be null), element types as given
void launch_axpy3(int64_t n, VecT in, VecT out_t, double a, const void* x, double b, const void* y,
                  double c, const void* z, void* out, hipStream_t s);
void launch_cast_f64_f32(const double* in, float* out, int64_t n, hipStream_t s);
void launch_cast_f32_f64(const float* in, double* out, int64_t n, hipStream_t s);

// Gram-Schmidt kernels (blas.hip)
struct Cgs2Ws {
    double* partial = nullptr;   // (JMAX_ALL + 2) * nb
    double* h1 = nullptr;        // JMAX_ALL
    double* h2 = nullptr;        // JMAX_ALL
    double* scal = nullptr;      // [0] = ||w_in||^2, [1] = ||w_out||^2, [2] = 1/beta
    double* t = nullptr;         // n
    double* dred = nullptr;      // delayed form: reduced inner products (2 JMAX_ALL + 3)
    double* coef = nullptr;      // delayed form: a, g (JMAX_ALL each) and 4 scalars
    int nb = 0;                  // blocks of the streaming kernels
    int nbf = 0;                 // blocks of the fused update-projection kernel
    int nbh = 0;                 // blocks of its half-row form (j > 32)
};
constexpr int CGS_JMAX_ALL = 256;
constexpr int CGS_JFUSED = 64;   // widest basis of the fused update-projection
int cgs_blocks(int64_t n);
// blocks of the Ritz-test inner products and residual norms (more than the
// Gram-Schmidt kernels': these read many vectors per row with few waves)
int ritz_blocks(int64_t n);
void carve_cgs2(Carver& c, int64_t n, Cgs2Ws& ws);
// Orthogonalise w against V[:, 0:j] (CGS2).  Writes the unnormalised result to
// w_out (may equal w), the Hessenberg column (j+1 entries: h, beta) to
// Hcol_d (device), and 1/beta (0 on breakdown) to ws.scal[2].  If v_next is
// non-null it receives w_out * (1/beta).
// G = V^T W: j x ncols, column-major on the device (V and W share the
// leading dimension ldv); one projection pass over V per column of W, the
// same two-stage reduction as the Gram-Schmidt kernels.
void launch_gram(int64_t n, int j, const double* V, int64_t ldv, const double* W, int ncols,
                 double* G_d, Cgs2Ws& ws, hipStream_t s);
void launch_cgs2(int64_t n, int j, const double* V, int64_t ldv, const double* w, double* w_out,
                 double* Hcol_d, double* v_next, double breakdown_tol, Cgs2Ws& ws,
                 hipStream_t s);

// Arnoldi with delayed reorthogonalisation (one block of inner products per
// step).  Step kinds, with Q = V[:, 0:jq] and H column-major (ld ldh):
//   DCGS_FIRST   z = w (= op(q_{jq-1})): h = Q^T z -> H[:, jq-1] (provisional),
//                u_out = z - Q h;
//   DCGS_LAGGED  u = candidate for q_jq, w = op(u): a = Q^T u finishes
//                H[:, jq-1] and q_jq -> q_out; op(q_jq)'s first pass gives
//                H[:, jq] (provisional) and the next candidate u_out;
//   DCGS_LAST    u = candidate for q_jq (no w): finishes H[:, jq-1] and q_jq.
// ws.scal[0] carries ||h||^2 of the provisional column between steps.
enum { DCGS_FIRST = 0, DCGS_LAGGED = 1, DCGS_LAST = 2 };
void launch_dcgs_step(int kind, int64_t n, int jq, const double* V, int64_t ldv, const double* u,
                      const double* w, double* Hd, int64_t ldh, double* q_out, double* u_out,
                      double breakdown_tol, Cgs2Ws& ws, hipStream_t s);

// C = V Q  (V n x kin, Q device kin x kout col-major ld kin) -- MFMA FP64
void launch_gemm_tall(int64_t n, int kin, int kout, const double* V, int64_t ldv,
                      const double* Q_d, double* C, int64_t ldc, hipStream_t s);

// Several dot products <a_i, b_i> of n-vectors, deterministic.
constexpr int MAX_DOTS = 64;
struct DotList {
    const double* a[MAX_DOTS];
    const double* b[MAX_DOTS];
    int count;
};
void launch_dots(int64_t n, const DotList& L, double* partial, int nb, double* out_d,
                 hipStream_t s);
// Norms^2 of linear combinations sum_t c_t v_t (up to 3 terms each).
constexpr int MAX_COMBOS = 32;
struct ComboList {
    const double* v[MAX_COMBOS][3];
    double c[MAX_COMBOS][3];
    int count;
};
void launch_combo_norms(int64_t n, const ComboList& L, double* partial, int nb, double* out_d,
                        hipStream_t s);
void launch_copy_cols_complex(int64_t n, const double* Y, int64_t ldy, const int* colmap_re,
                              const int* colmap_im, const double* scale, int ncols,
                              double* X, hipStream_t s);
void launch_zero(double* p, int64_t count, hipStream_t s);

// ---------------------------------------------------------------- host LA
// Real nonsymmetric eigenproblem of a small dense matrix (column-major).
// Eigenvalues: conjugate pairs adjacent, Im > 0 first.  Vectors optional.
void dense_eig(int n, const double* a, std::vector<cplx>& w, std::vector<cplx>* V);
// Eigenvalues of an upper Hessenberg matrix (column-major), no vectors.
void hessenberg_eigvals(int n, std::vector<double>& h, std::vector<cplx>& w);
// Solve M x = b by Gaussian elimination with partial pivoting (column-major).
bool lu_solve(int n, std::vector<double> M, std::vector<double>& b);
// Orthonormal basis of the columns of B (m x k, column-major), Householder QR.
void orthonormal_basis(int m, int k, const std::vector<double>& B, std::vector<double>& Q);

// ---------------------------------------------------------------- method
std::vector<cplx> harmonic_ritz(int d, const std::vector<double>& Hbar /*(d+1) x d col-major*/);
std::vector<cplx> leja_order(const std::vector<cplx>& theta);
// Apply pi(A) (or pi_2(tau(A))) to v: FP64 or FP32 chain.
struct ApplyWs {
    void* buf[8] = {};   // n-vectors of the chain's element type (apply_buffers of them)
};
int apply_buffers(const Poly& p);
void carve_apply(Carver& c, int64_t n, const Poly& p, VecT t, ApplyWs& ws);
// in/out types: vin/vout select the element type of v and y; the chain runs in
// `chain` precision (F32 chain = FP32 matrix values).
// Stability control of section 7 (host): log10 pof per root, the number of
// extra copies per root, and the root list with the copies placed.
std::vector<double> log10_pof(const std::vector<cplx>& th);
std::vector<int> extra_root_counts(const std::vector<cplx>& th);
std::vector<cplx> add_stability_roots(const std::vector<cplx>& th, int* added);

// Algorithmic bytes of the fused SpMV passes of one apply_poly with chain
// element type `chain` (nothing is launched).
size_t apply_poly_bytes(const Matrix& A, const Poly& p, VecT chain);
// Returns the algorithmic bytes of its fused SpMV passes.
size_t apply_poly(const Matrix& A, const Poly& p, VecT vin, const void* v, VecT vout, void* y,
                  VecT chain, ApplyWs& ws, hipStream_t s);
// y = c * pi(A) v + gamma z for a single root list, all FP64 (the operator
// tau(A) = I - pi_1(A) of section 8 is c = -1, gamma = 1, z = v).
size_t apply_single_epilogue(const Matrix& A, const std::vector<cplx>& roots, const double* v,
                             double* y, double c, double gamma, const double* z, ApplyWs& ws,
                             hipStream_t s, double sigma = 0.0);
// ---------------------------------------------------------------- projected problem (ritz.cpp)
// Ordering of Ritz values (section 4): increasing |target - nu|, ties larger
// Im first, then smaller Re.  target = 1 for pi(A), 0 for A itself.
std::vector<int> sort_ritz(const std::vector<cplx>& nu, double target);
struct RitzPlan {
    int mc = 0, nw = 0;
    std::vector<cplx> nu;        // sorted Ritz values of the operator (mc)
    std::vector<cplx> G;         // mc x mc eigenvectors of H_m, sorted columns
    std::vector<int> cre, cim;   // wanted i: columns of Y holding Re / Im of y_i (cim = -1: real)
    std::vector<int> dup;        // wanted i is the conjugate of wanted i-1 (same columns)
    int ycols = 0;
    std::vector<double> Gw;      // mc x ycols: Y = V_m Gw
    bool harmonic = false;       // harmonic Ritz pairs (then fh, hm are set)
    std::vector<double> fh;      // f = (H_m - target I)^{-T} e_m
    double hm = 0.0;             // h_{m+1,m}
};
// Ritz pairs of H_m, or with `harmonic` (and hm != 0) the harmonic Ritz pairs
// with respect to `target`: eig(H_m + hm^2 f e_m^T), f = (H_m - target I)^{-T} e_m.
RitzPlan plan_ritz(const std::vector<double>& Hm, int mc, int nev, double target,
                   bool harmonic = false, double hm = 0.0);
// Ritz-test dot products: kind 0 is y_a . (A y)_b, kind 1 is y_a . y_b.
struct DotSpec {
    int a, b, kind;
};
std::vector<DotSpec> ritz_dots(const RitzPlan& R);
void ritz_mu(const RitzPlan& R, const std::vector<double>& dv, std::vector<cplx>& mu,
             std::vector<double>& ynorm);
// ||sum_t c_t v_t||^2 with v_t column col[t] of AY (kind 0) or Y (kind 1).
struct ComboSpec {
    int owner;
    int col[3];
    int kind[3];
    double c[3];
    int nterms;
};
std::vector<ComboSpec> ritz_combos(const RitzPlan& R, const std::vector<cplx>& mu);
void ritz_resid(const RitzPlan& R, const std::vector<ComboSpec>& cs, const std::vector<double>& rn,
                const std::vector<double>& ynorm, std::vector<double>& res);
int64_t ritz_mvps(const RitzPlan& R);
struct RestartPlan {
    int kk = 0;
    std::vector<double> Q;    // mc x kk orthonormal basis of the kept Ritz vectors
    std::vector<double> Qp;   // (m+1) x (kk+1): [[Q, 0], [0, 1]]
    std::vector<double> Hn;   // (m+1) x m: new projected matrix (first kk columns)
};
RestartPlan plan_restart(const RitzPlan& R, const std::vector<double>& Hm, double hm, int m, int k);

// Mixed precision (FP32 pi(A)v, FP64 elsewhere), shared by the single-solve
// driver and the batched engine.  leave_fp32: after an FP32 cycle whose
// largest wanted residual is hist.back() (hist: one maximum per cycle so far),
// whether the FP32 phase ends: the residuals reached the FP32 floor
// 100 eps_32 ||A||, or stopped improving (less than 2x over two cycles) within
// three decades of it.
bool leave_fp32(const std::vector<double>& hist, double anorm);

// polynomial construction and Arnoldi drivers (eigs.cpp)
size_t poly_build_ws(int64_t n, int d, bool dbl);
int poly_build(const Matrix& A, int d1, int d2, const double* b, void* ws, size_t ws_bytes,
               hipStream_t s, Poly& out, double sigma = 0.0, bool lowsync = false);
size_t eigs_ws(const Matrix& A, const Poly* p, const ppa_eigs_opts& o);
size_t poly_build_ex_ws(const Matrix& A, const ppa_poly_build_opts& o, bool two);
int poly_build_ex(const Matrix& A, const ppa_poly_build_opts& o, const double* b, const double* b2,
                  void* ws, size_t ws_bytes, hipStream_t s, Poly& out, ppa_poly_build_info& info);
int eigs(const Matrix& A, const Poly* p, const ppa_eigs_opts& o, const double* v0, void* ws,
         size_t ws_bytes, hipStream_t s, ppa_eigs_result& r);

// ---------------------------------------------------------------- batched engine (batch.hip)
struct Batch;
// nnz and precision (PPA_F64 or PPA_MIXED) matter only for PPA_MIXED: room
// for the FP32 values and the FP32 chain vectors.
size_t batch_ws_bytes(int64_t n, int d, int m, int nev, int64_t nnz = 0, int precision = PPA_F64);
Batch* batch_create(int max_slots, hipStream_t s);
void batch_destroy(Batch* B);
int batch_submit(Batch& B, const ppa_batch_request& rq, int* slot, int precision = PPA_F64);
int batch_step(Batch& B, int* finished, int cap, int* nfin, int* nactive);
int batch_result(Batch& B, int slot, ppa_eigs_result& r);

}  // namespace ppa
