/*
 * ppa.h -- C ABI of libppa.so, polynomial preconditioned Arnoldi on one
 * MI355X (gfx950).  Method: Embree, Loe & Morgan, "Polynomial Preconditioned
 * Arnoldi" (arXiv:1806.08020).
 *
 * Conventions
 *  - Pointers named *_d are device pointers (HIP global memory on the current
 *    device); all other pointers are host pointers.
 *  - The library never takes ownership of caller memory.  Device arrays passed
 *    to ppa_matrix_create are borrowed for the lifetime of the handle.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is enqueued on it; calls documented as synchronising wait for it.
 *  - Scratch device memory on the solve paths comes from a caller-provided
 *    workspace (`ws_d`, `ws_bytes`), sized by the *_workspace_bytes queries;
 *    those paths never call hipMalloc.  Handle creation may allocate.
 *  - Vectors are contiguous; a block of vectors is column-major with leading
 *    dimension n unless stated otherwise.
 *  - Every entry point returns a ppa_status.  On a negative status nothing was
 *    written to the outputs and ppa_last_error() (thread-local) describes the
 *    failure; positive statuses are warnings and the outputs are filled.
 *  - A handle is used by one host thread at a time; distinct handles may be
 *    used concurrently from different threads.
 */
#ifndef PPA_H
#define PPA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PPA_ABI_VERSION 1

typedef enum ppa_status {
    PPA_OK = 0,
    PPA_WARN_DEGREE_REDUCED = 1,  /* GMRES broke down early: lower-degree polynomial */
    PPA_WARN_NOT_CONVERGED = 2,   /* max_cycles reached; best estimates returned   */
    PPA_WARN_BREAKDOWN = 3,       /* Arnoldi basis became invariant; see result     */
    PPA_ERR_INVALID = -1,         /* bad argument or malformed matrix               */
    PPA_ERR_HIP = -2,             /* a HIP runtime call failed                      */
    PPA_ERR_WORKSPACE = -3,       /* workspace missing or too small                 */
    PPA_ERR_NONFINITE = -4,       /* NaN/Inf met in the input or during the solve   */
    PPA_ERR_SINGULAR = -5,        /* H_d singular in the harmonic Ritz solve        */
    PPA_ERR_NUMERIC = -6,         /* small dense eigensolver did not converge       */
    PPA_ERR_BUSY = -7             /* batched engine: no free slot                   */
} ppa_status;

typedef enum ppa_precision {
    PPA_F64 = 0,    /* everything in FP64                                           */
    PPA_F32 = 1,    /* pi(A)v with FP32 matrix values and FP32 vectors              */
    PPA_MIXED = 2   /* eigs: pi(A)v in FP32, orthogonalisation / Ritz / residual in
                       FP64; when the FP32 cycles stall, a closing FP64
                       Rayleigh-Ritz with A on their basis, then, unless it
                       already meets rtol, FP64 cycles from v0 again         */
} ppa_precision;

typedef struct ppa_matrix ppa_matrix;
typedef struct ppa_poly ppa_poly;

/* ABI version (PPA_ABI_VERSION) and the last error message of this thread. */
int ppa_abi_version(void);
const char* ppa_last_error(void);

/* ------------------------------------------------------------------------
 * Sparse matrix A (section 4: A is large, sparse, possibly nonsymmetric; the
 * paper's cost model counts nnzr nonzeros per row).
 *
 * n           number of rows = columns (1 <= n < 2^31)
 * rowptr_d    int32[n+1], rowptr_d[0] = 0, nondecreasing
 * colind_d    int32[nnz], column indices in [0, n), strictly increasing in a row
 * val64_d     double[nnz] values (required)
 * val32_d     float[nnz] values for the FP32 / mixed paths, or NULL.  When NULL
 *             and flags has PPA_MATRIX_F32, the library converts val64_d into
 *             an internal FP32 copy it owns.
 * flags       PPA_MATRIX_* bits.
 * stream      stream used for validation and tuning; the call synchronises it.
 * out         receives the handle.
 *
 * Validates the CSR structure on the device (PPA_ERR_INVALID if malformed),
 * computes ||A||_inf, and builds the row-block partitions used by the SpMV
 * kernels (allocated by the library, freed by ppa_matrix_destroy).  For large
 * matrices (n >= 200000, nnz >= 10^6) whose row blocks touch narrow column
 * ranges and whose tuned plain pass runs below half the HBM peak (4 TB/s) it
 * also times the LDS-windowed and sliding-window SpMVs against the plain one
 * and keeps the fastest (a staged variant only for a 5% gain); all
 * sum each row in column order, so they agree bitwise on every row that fits
 * one block of the plain kernel's block shape (2048 or 256 nonzeros, see
 * ppa_matrix_spmv_blocks); longer rows are tree-reduced by the plain kernel
 * and agree to rounding.
 * ------------------------------------------------------------------------ */
#define PPA_MATRIX_F32 1            /* build an FP32 copy of the values           */
#define PPA_MATRIX_WINDOW_FORCE 2   /* use the windowed SpMV whenever it fits     */
#define PPA_MATRIX_WINDOW_OFF 4     /* never use a windowed SpMV (either kind)    */
#define PPA_MATRIX_RING_FORCE 8     /* use the sliding-window SpMV whenever it fits
                                       (not with PPA_MATRIX_WINDOW_FORCE)         */
#define PPA_MATRIX_NO_TUNE 16       /* no timing at creation: the size rule's cache
                                       policy, large blocks, no staged variant
                                       unless forced (for matrices used briefly,
                                       where the timing would not pay)           */
#define PPA_MATRIX_RUNS_FORCE 32    /* build the column runs of the plain kernel's
                                       large blocks and use them (both value
                                       types), see ppa_matrix_spmv_runs          */
#define PPA_MATRIX_TWO_STEP 64      /* build the records for two factors of pi per
                                       pass where the bandwidth allows it, and
                                       use them, see ppa_matrix_two_step         */
int ppa_matrix_create(int64_t n, const int32_t* rowptr_d, const int32_t* colind_d,
                      const double* val64_d, const float* val32_d, int flags,
                      void* stream, ppa_matrix** out);
int ppa_matrix_destroy(ppa_matrix* A);
/* n, nnz, ||A||_inf (largest absolute row sum) and the number of row blocks. */
int ppa_matrix_info(const ppa_matrix* A, int64_t* n, int64_t* nnz, double* norm_inf,
                    int64_t* nblocks);
/* SpMV variant in use for FP64 (precision PPA_F64) or FP32 (PPA_F32) values:
 * *windowed = 0 for the plain kernel, 1 for the LDS-windowed one (each row
 * block stages its column range of u in LDS), 2 for the sliding-window one
 * (one persistent block per CU walks consecutive row chunks and keeps u in
 * an LDS ring, loading only the columns each chunk adds; band matrices).
 * All three sum each row in column order. */
int ppa_matrix_spmv_variant(const ppa_matrix* A, int precision, int* windowed);

/* Cache policy of the plain (non-windowed) SpMV kernel, per value precision
 * (PPA_F64 or PPA_F32).  It changes how the kernel's loads and stores treat
 * the caches, never the arithmetic: every policy gives bitwise identical
 * results.
 *   PPA_CACHE_STREAM     non-temporal loads of column indices and values;
 *   PPA_CACHE_KEEP       plain loads and stores, so that a matrix that fits in
 *                        the 256 MB last-level cache stays there from one
 *                        factor of pi to the next;
 *   PPA_CACHE_KEEP_NTST  plain loads, non-temporal stores of the output.
 * ppa_matrix_create picks KEEP when one pass moves at most 128 MB and STREAM
 * otherwise, and on large matrices (n >= 200000, nnz >= 10^6) times the
 * three (with both block shapes, ppa_matrix_spmv_blocks) and switches only
 * when another is at least 3% faster.  The setter overrides that choice
 * (PPA_ERR_INVALID for an unknown policy or precision, or PPA_F32 without
 * FP32 values); it must not race with launches that use A. */
#define PPA_CACHE_STREAM 0
#define PPA_CACHE_KEEP 1
#define PPA_CACHE_KEEP_NTST 2
int ppa_matrix_cache_policy(const ppa_matrix* A, int precision, int* policy);
int ppa_matrix_set_cache_policy(ppa_matrix* A, int precision, int policy);

/* Block shape of the plain SpMV kernel, per value precision: *nnz_per_block
 * = 2048 (blocks of 256 threads, the default) or 256 (blocks of 64
 * threads).  Both sum each row in column order, so they agree bitwise on
 * rows of at most 256 nonzeros; longer rows are reduced across a block in
 * the small shape and agree to rounding.  ppa_matrix_create times both
 * shapes with the cache policies on large matrices and switches only for a
 * 3% gain; the setter overrides (PPA_ERR_INVALID for another value). */
int ppa_matrix_spmv_blocks(const ppa_matrix* A, int precision, int* nnz_per_block);
int ppa_matrix_set_spmv_blocks(ppa_matrix* A, int precision, int nnz_per_block);

/* Column runs of the plain kernel (large blocks).  The columns one row block
 * gathers form a few contiguous runs for stencil and band matrices (a 3-D
 * 7-point stencil: three runs, the planes below and above and the rows
 * around the block).  With runs on, each block copies its runs of the
 * gathered vector into LDS with 16-byte loads issued together with the
 * matrix stream, so no gather waits for a column index to arrive from
 * memory; blocks with more than 7 runs, or more than 10 KB of them in the
 * value type, gather from memory as without.  Results are bitwise those of
 * the plain kernel.  The runs are built at creation by PPA_MATRIX_RUNS_FORCE
 * or by the creation timing on large matrices (which then times them with
 * the three cache policies and keeps them only for a 3% gain).
 * *on receives 1 when the plain kernel of `precision` uses them.  The setter
 * turns them on (1; the large block shape is then used) or off (0);
 * PPA_ERR_INVALID when they were not built.  It must not race with launches
 * that use A.  *blocks_with_runs (may be NULL) receives how many large blocks
 * have runs that fit the LDS budget of that value type. */
int ppa_matrix_spmv_runs(const ppa_matrix* A, int precision, int* on, int64_t* blocks_with_runs);
int ppa_matrix_set_spmv_runs(ppa_matrix* A, int precision, int on);

/* Two factors of pi per pass (a matrix-powers form of eq. (2.1), section 9
 * names communication-avoiding variants): for a matrix whose entries all
 * lie within h of the diagonal, one block per CU owns a range of output
 * rows, stages the gathered vector on that range widened by 2h in LDS,
 * computes the first of two consecutive factors on the range widened by h
 * into LDS and the second on its own rows from there.  The polynomial
 * application (ppa_poly_apply, and the Arnoldi cycles of ppa_eigs) then
 * takes two real roots in a row, or a conjugate pair, in one launch, except
 * for the last factor; every result is bitwise that of the single passes.
 * The matrix is read on each block's rows widened by h and again on its own
 * rows, and the intermediate vector never reaches memory; where the form
 * fits, a CU's row range is so short against 2h that this saves only that
 * vector's store and reload, and the form can be slower than the single
 * passes, so it is used only on request.  The records are built at creation by
 * PPA_MATRIX_TWO_STEP when no row has more than 2048 nonzeros and a
 * block's ranges fit its LDS (FP64: (2R + 6h + 4096) * 8 bytes <= 160 KB,
 * R = n / CUs; FP32 half that).  *on receives 1 when the form is in use for
 * `precision`, *bandwidth the h found (-1 when no records were built; both
 * may be NULL).  The setter turns it on (1) or off (0); PPA_ERR_INVALID when
 * it does not fit that value type.  It must not race with launches that
 * use A. */
int ppa_matrix_two_step(const ppa_matrix* A, int precision, int* on, int* bandwidth);
int ppa_matrix_set_two_step(ppa_matrix* A, int precision, int on);

/* ------------------------------------------------------------------------
 * Polynomial pi in factored form, eq. (2.1): pi(z) = prod_i (1 - z/theta_i),
 * roots in modified Leja order with each complex root followed at once by its
 * conjugate (section 2, step 1(c); section 7: keep complex roots together).
 * A double polynomial (section 8) is pi_2(tau(z)), tau = 1 - pi_1.
 * ------------------------------------------------------------------------ */

/* Polynomial from given roots (host arrays re[deg], im[deg]), used in the
 * given order.  A root with im != 0 must be followed by its exact conjugate.
 * d1 = 0: single polynomial with roots (re, im).  d1 > 0: double polynomial,
 * (re1, im1)[d1] are the roots of pi_1 and (re, im)[deg] those of pi_2. */
int ppa_poly_from_roots(int deg, const double* re, const double* im,
                        int d1, const double* re1, const double* im1, ppa_poly** out);
int ppa_poly_destroy(ppa_poly* p);
/* Degrees: *deg = degree of pi (or pi_2), *d1 = degree of pi_1 (0 if single). */
int ppa_poly_degree(const ppa_poly* p, int* deg, int* d1);
/* Copy roots of level 2 (pi, or pi_2 of a double polynomial) or level 1 (pi_1)
 * into host arrays of capacity `cap`; returns the count in *count. */
int ppa_poly_roots(const ppa_poly* p, int level, double* re, double* im, int cap, int* count);

/* Stability control (section 7, "Adding roots for stability").
 * ppa_poly_log10_pof: log10 pof(j) for every root theta_j of `level` (2: pi,
 * or pi_2 of a double polynomial; 1: pi_1), in application order, where
 * pof(j) = prod_{i != j} |1 - theta_j / theta_i| (so |pi'(theta_j)| =
 * pof(j) / |theta_j|; -inf for a repeated root).  `out` holds `cap` doubles;
 * *count receives the root count.  Host only.
 * ppa_poly_stabilize: a new polynomial equal to p except that every root of
 * `level` with pof(j) > 1e4 gets ceil((log10 pof(j) - 4) / 14) extra copies
 * (a double root above 1e4, triple above 1e18, ...).  The first copy goes to
 * the end of the root list, the others are spaced evenly between the root
 * and the end; a conjugate pair is copied as a pair and never split
 * (section 8, Example 9 applies the same test to pi_2).  *added receives the
 * number of roots added; the caller destroys *out.  Host only. */
int ppa_poly_log10_pof(const ppa_poly* p, int level, double* out, int cap, int* count);
int ppa_poly_stabilize(const ppa_poly* p, int level, ppa_poly** out, int* added);

/* Workspace bytes for ppa_poly_build / ppa_poly_build_double with degree d
 * (for a double polynomial pass d = max(d1, d2) and double_poly = 1). */
int ppa_poly_build_workspace_bytes(const ppa_matrix* A, int d, int double_poly, size_t* bytes);

/* GMRES polynomial (section 2, step 1): one cycle of GMRES(d) on A from b_d
 * (double[n], device; need not be normalised) with classical Gram-Schmidt and
 * one reorthogonalisation pass on the device; harmonic Ritz values
 * theta = eig(H_d + h_{d+1,d}^2 f e_d^T), f = H_d^{-T} e_d (step 1(b)) and
 * modified Leja ordering (step 1(c)) on the host in FP64.  Synchronises
 * `stream`.  If the Krylov space becomes invariant at step j < d the degree is
 * reduced to j and PPA_WARN_DEGREE_REDUCED is returned. */
int ppa_poly_build(const ppa_matrix* A, int d, const double* b_d,
                   void* ws_d, size_t ws_bytes, void* stream, ppa_poly** out);

/* Double polynomial (section 8): pi_1 of degree d1 from GMRES on A, then pi_2 of
 * degree d2 from GMRES on tau(A) = I - pi_1(A), both started from b_d. */
int ppa_poly_build_double(const ppa_matrix* A, int d1, int d2, const double* b_d,
                          void* ws_d, size_t ws_bytes, void* stream, ppa_poly** out);

/* Polynomial-quality safeguards (sections 5 and 6).
 *   d        requested degree.
 *   damp     GMRES start vector A^damp b (0, 1 or 2): premultiplying by A damps
 *            b's components along eigenvectors of small eigenvalues (section 6).
 *   alpha    when nonzero and damp >= 1, alpha * b is added on the last
 *            product (the A b + alpha b family of section 6).
 *   test_m, test_k, test_nev
 *            0: no test.  Otherwise the Ideal-Order-Condition heuristic of
 *            section 6: one Arnoldi(test_m, test_k) cycle on pi(A) from b,
 *            Ritz values ordered by |1 - nu|, Rayleigh quotients mu_j = y_j^* A y_j
 *            of the first test_k, and the condition |mu_1| <= ... <= |mu_nev| <
 *            min_{nev < j <= k} |mu_j|.  If it fails the start vector is damped
 *            once more (A b in place of b, up to damp = 2); while it still fails
 *            the degree is halved, down to 1.  Needs 1 <= test_nev <= test_k <
 *            test_m <= 64, test_k <= 32, n > test_m. */
typedef struct {
    int d;
    int damp;
    double alpha;
    int test_m, test_k, test_nev;
    double shift;   /* target mu (section 2 footnote): the polynomial is built for
                       and applied to A - mu I; the order test and ppa_eigs then
                       rank eigenvalues by their distance to mu (0: the origin) */
    int flags;      /* PPA_FLAG_LOWSYNC: the delayed-reorthogonalisation Gram-
                       Schmidt in the GMRES cycle and the order test; 0 otherwise */
} ppa_poly_build_opts;

typedef struct {
    int degree;     /* degree of the returned polynomial                       */
    int damp;       /* damping power of its start vector                       */
    int attempts;   /* polynomials built                                        */
    int held;       /* 1/0: the Ideal Order Condition held / failed for it;
                       -1: not tested                                          */
} ppa_poly_build_info;

/* The target mu of a polynomial: it acts on A - mu I (set by
 * ppa_poly_build_ex; 0 for the other builders).  ppa_poly_set_shift sets it
 * on a polynomial whose roots were computed for A - mu I (ppa_poly_from_roots).
 * ppa_eigs with such a polynomial iterates on pi(A - mu I), tests and
 * returns Rayleigh quotients of A itself (the residual A y - lam y is the
 * same for both) ordered by distance to mu.  Real mu only. */
int ppa_poly_shift(const ppa_poly* p, double* shift);
int ppa_poly_set_shift(ppa_poly* p, double shift);

/* Workspace bytes of ppa_poly_build_ex (two_start: b2_d will be given). */
int ppa_poly_build_ex_workspace_bytes(const ppa_matrix* A, const ppa_poly_build_opts* o,
                                      int two_start, size_t* bytes);

/* GMRES polynomial with the safeguards above.  b_d: double[n] start vector.
 * b2_d: NULL, or a second start vector (section 5, "polynomial determined by
 * two starting vectors"): GMRES(d) then runs on the block-diagonal system
 * diag(A, A) of dimension 2n from [b; b2] with each half scaled to norm
 * 1/sqrt(2), and its polynomial is returned (damping applies to both
 * vectors; the order test cycle starts from b_d).  *info receives what was
 * done.  Synchronises `stream`.  Returns PPA_WARN_DEGREE_REDUCED as
 * ppa_poly_build does. */
int ppa_poly_build_ex(const ppa_matrix* A, const ppa_poly_build_opts* o, const double* b_d,
                      const double* b2_d, void* ws_d, size_t ws_bytes, void* stream,
                      ppa_poly** out, ppa_poly_build_info* info);

/* Workspace bytes for ppa_poly_apply. */
int ppa_poly_apply_workspace_bytes(const ppa_matrix* A, const ppa_poly* p, int precision,
                                   size_t* bytes);

/* y = pi(A) v (eq. (2.1); section 8 for a double polynomial).
 * precision PPA_F64: v_d, y_d are double[n]; PPA_F32: float[n] and the FP32
 * matrix values are used (the handle must hold them).  v_d and y_d must not
 * alias.  Each real root costs one fused pass y = w - (1/theta) A w over the
 * CSR arrays; a conjugate pair a +/- ib costs two: s = 2a w - A w and
 * y = w - A s / (a^2 + b^2).  Asynchronous on `stream`. */
int ppa_poly_apply(const ppa_matrix* A, const ppa_poly* p, int precision,
                   const void* v_d, void* y_d, void* ws_d, size_t ws_bytes, void* stream);

/* Size of the static device array behind ppa_poly_apply_noalloc (64 MiB). */
#define PPA_NOALLOC_SCRATCH_BYTES (64u << 20)

/* y = pi(A) v as ppa_poly_apply, for callers that cannot allocate device
 * memory and cannot bring a workspace (code under HIP graph capture, tight
 * serving loops, hosts that forbid hipMalloc).  The chain's temporaries
 * (ppa_poly_apply_workspace_bytes of them) live in a static device array of
 * PPA_NOALLOC_SCRATCH_BYTES per device, which the library holds until the
 * process ends; the call allocates nothing.  Same kernels and results as
 * ppa_poly_apply.  Limits: the workspace must fit the array (FP64: 4 n-vectors
 * for a single polynomial, 6 for a double one, 7 for a shifted double one;
 * FP32 half the bytes), else PPA_ERR_WORKSPACE and nothing is launched.
 * The current device must be the matrix's.  Every call on one device shares
 * that device's array: calls that overlap on one device (two streams, or two
 * host threads) race on it and must be serialised by the caller.
 * Asynchronous on `stream`; the first call on a device looks the array's
 * device address up (hipGetSymbolAddress). */
int ppa_poly_apply_noalloc(const ppa_matrix* A, const ppa_poly* p, int precision,
                           const void* v_d, void* y_d, void* stream);

/* Algorithmic HBM bytes of one ppa_poly_apply in `precision`, summed over its
 * fused passes: the CSR arrays once per pass (values, int32 column indices,
 * int32 row pointers), each distinct input vector once and the output once.
 * A real root moves 2 vectors, a conjugate pair 2 + 3.  Host only: launches
 * nothing. */
int ppa_poly_apply_bytes(const ppa_matrix* A, const ppa_poly* p, int precision, double* bytes);

/* One fused pass, the building block of ppa_poly_apply:
 *   out = alpha x + beta (A u) + gamma z + delta z2
 * (x, z, z2 may be NULL, dropping their term).  Types: in_f32 selects
 * float for x, u, z, z2 (else double); out_f32 float for out (else double);
 * FP32 matrix values are used iff in_f32 || out_f32.  out must not alias u. */
int ppa_fused_spmv(const ppa_matrix* A, int in_f32, int out_f32, double alpha,
                   const void* x_d, double beta, const void* u_d, double gamma,
                   const void* z_d, double delta, const void* z2_d, void* out_d,
                   void* stream);

/* ------------------------------------------------------------------------
 * Classical Gram-Schmidt with one reorthogonalisation pass (section 4: every
 * projection step is repeated once against the same basis).
 *   V_d  double, n x (j) column-major, leading dimension ldv >= n, orthonormal
 *   w_d  double[n] (overwritten with the orthogonalised, unnormalised vector)
 *   h    host double[j+1]: h[0..j-1] = V^T w over both passes, h[j] = ||w_out||
 *   w0norm host double: ||w_in||.
 * Synchronises `stream`.
 * ------------------------------------------------------------------------ */
int ppa_cgs2_workspace_bytes(int64_t n, int j, size_t* bytes);
int ppa_cgs2(int64_t n, int j, const double* V_d, int64_t ldv, double* w_d,
             double* h, double* w0norm, void* ws_d, size_t ws_bytes, void* stream);

/* Dense tall-skinny product C = V Q (the thick-restart update V_k = V_m Q of
 * section 4 and the Ritz vectors Y = V_m G), on MFMA FP64.
 *   V_d double n x kin (ld ldv), Q host double kin x kout (column-major,
 *   ld kin), C_d double n x kout (ld ldc), C must not overlap V.
 * kin <= 128, kout <= 64.  Asynchronous on `stream` (Q is staged through the
 * workspace, ppa_gemm_workspace_bytes). */
int ppa_gemm_workspace_bytes(int kin, int kout, size_t* bytes);
int ppa_gemm_tall(int64_t n, int kin, int kout, const double* V_d, int64_t ldv,
                  const double* Q, double* C_d, int64_t ldc, void* ws_d, size_t ws_bytes,
                  void* stream);

/* ------------------------------------------------------------------------
 * Thick-restarted Arnoldi(m, k) on pi(A) (section 2 step 2, section 4).
 * ------------------------------------------------------------------------ */
typedef struct ppa_eigs_opts {
    int m;            /* largest subspace dimension, 2 <= m <= 64            */
    int k;            /* Ritz vectors kept at a restart, nev <= k < m        */
    int nev;          /* wanted eigenpairs, 1 <= nev                          */
    int max_cycles;   /* restart cycles allowed (>= 1)                        */
    double rtol;      /* converged when ||A y - mu y|| <= rtol * anorm        */
    double anorm;     /* norm used with rtol; <= 0 selects ||A||_inf          */
    int precision;    /* PPA_F64 or PPA_MIXED                                 */
    int flags;        /* PPA_FLAG_* bits                                      */
} ppa_eigs_opts;

/* opts.flags: time the polynomial applications and the orthogonalisation with
 * HIP events recorded on `stream` (results in t_apply_ms / t_cgs_ms). */
#define PPA_FLAG_TIMING 1
/* Harmonic restart (the harmonic Arnoldi variant of section 4, Example 2):
 * each cycle takes harmonic Ritz pairs of the operator with respect to its
 * target (1 for pi(A), 0 without a polynomial), eig(H_m + h^2 f e_m^T) with
 * (H_m - target I)^T f = e_m, tests them as usual, and restarts with the
 * kept harmonic Ritz vectors plus v_{m+1} - h V_m f, whose direction all
 * their residuals share. */
#define PPA_FLAG_HARMONIC 2
/* Low-synchronisation Gram-Schmidt: the reorthogonalisation pass of step j-1
 * is delayed and merged with the projection of step j, so each Arnoldi step
 * makes two passes over the basis (one block of inner products, one update)
 * instead of three.  The operator acts on the once-orthogonalised candidate;
 * op(q_j)'s projection follows from op(Q) a = V_{j+1} Hbar a.  Same Arnoldi
 * decomposition as the default in exact arithmetic (a form of section 4's
 * Gram-Schmidt with reorthogonalisation; section 9 names communication-
 * avoiding variants as future work). */
#define PPA_FLAG_LOWSYNC 4
/* Record each restart cycle's Krylov steps (operator applications and
 * Gram-Schmidt: every launch between two host synchronisations) into a HIP
 * graph on a private capture stream, and replay it on `stream` whenever a
 * later cycle starts from the same column with the same basis buffer and
 * operator precision (at most four graphs per solve; the restart alternates
 * two basis buffers).  The launches are the same, so results are bitwise
 * those of the eager run; replays save the per-launch host overhead, which
 * dominates for small and mid-size matrices.  Ignored with PPA_FLAG_TIMING. */
#define PPA_FLAG_GRAPH 8

typedef struct ppa_eigs_result {
    /* host arrays of capacity nev, filled with the returned pairs sorted by
     * |mu| (ties: real part, then imaginary part) */
    double* lam_re;
    double* lam_im;
    double* resid;       /* ||A y - mu y|| with unit y                       */
    double* ritz_re;     /* Ritz values nu of pi(A) for the same pairs (may be NULL);
                            a mixed solve that ends with its closing
                            Rayleigh-Ritz returns the Ritz values of A there */
    double* ritz_im;
    /* device array (may be NULL): n x nev complex128 (interleaved re, im),
     * column j the unit eigenvector estimate of lam j */
    double* X_d;
    /* outputs */
    int nconv;           /* returned pairs meeting the tolerance             */
    int cycles;          /* restart cycles run                               */
    int64_t mvps;        /* products with A (polynomial build excluded)      */
    int64_t dots;        /* inner products                                   */
    int64_t vops;        /* length-n vector operations                       */
    double max_resid;    /* largest residual among the returned pairs        */
    int fp32_cycles;     /* cycles run with FP32 pi(A)v (PPA_MIXED)          */
    int reserved;
    int64_t spmv_passes; /* fused SpMV passes issued by the operator applications */
    int64_t spmv_passes_f32; /* of which with FP32 values and vectors (PPA_MIXED) */
    double spmv_bytes;   /* algorithmic bytes of those passes: CSR arrays once, each
                            distinct input vector once, the output once, per pass */
    double t_apply_ms;   /* PPA_FLAG_TIMING: device time of all operator applications */
    double t_cgs_ms;     /* PPA_FLAG_TIMING: device time of all CGS2 steps   */
} ppa_eigs_result;

/* Workspace bytes for ppa_eigs. */
int ppa_eigs_workspace_bytes(const ppa_matrix* A, const ppa_poly* p, const ppa_eigs_opts* o,
                             size_t* bytes);

/* Polynomial preconditioned Arnoldi: the nev eigenpairs of A whose pi-images
 * lie nearest 1 (i.e. of smallest magnitude for a GMRES polynomial), tested on
 * A with Rayleigh quotients mu = y^* A y of unit Ritz vectors at the end of each
 * cycle (section 4).  A restart keeps k Ritz vectors, k-1 when the k-th and
 * (k+1)-th form a conjugate pair.  p == NULL runs standard Arnoldi on A and
 * orders Ritz values by |nu|.  v0_d: start vector double[n] (device).
 * Synchronises `stream` once per cycle.  Returns PPA_OK when all nev pairs
 * converged, PPA_WARN_NOT_CONVERGED after max_cycles (outputs hold the last
 * estimates), PPA_WARN_BREAKDOWN if the basis became invariant. */
int ppa_eigs(const ppa_matrix* A, const ppa_poly* p, const ppa_eigs_opts* o,
             const double* v0_d, void* ws_d, size_t ws_bytes, void* stream,
             ppa_eigs_result* r);

/* ------------------------------------------------------------------------
 * Batched engine for many small solves (the served form; section 2 algorithm
 * and section 4 Arnoldi(m,k) for each request).  One launch advances every
 * admitted solve by one phase -- GMRES(d) build, Krylov steps on pi(A) up to
 * a pass budget, or the Ritz test -- with one workgroup per solve and every
 * reduction inside that workgroup, so a solve's result does not depend on the
 * other solves in the batch.  The host handles the small projected problems
 * between launches.  Requests join free slots and leave between launches
 * (continuous batching).  FP64 throughout, or per request PPA_MIXED
 * (ppa_batch_submit_ex): pi(A)v in FP32 as in ppa_eigs, with the same rule
 * for leaving the FP32 phase and the same closing FP64 Rayleigh-Ritz pass.
 * No eigenvectors are returned.
 * ------------------------------------------------------------------------ */
typedef struct ppa_batch ppa_batch;

typedef struct ppa_batch_request {
    int64_t n;                /* rows of A (n > m, n > d)                        */
    const int32_t* rowptr_d;  /* CSR of A (device, borrowed until the result is taken) */
    const int32_t* colind_d;
    const double* val_d;
    double anorm;             /* norm for rtol; <= 0: ||A||_inf computed at submit */
    int d;                    /* GMRES polynomial degree, 1 <= d <= 126          */
    int m, k, nev;            /* Arnoldi(m,k), nev wanted; m <= 64, nev <= 32    */
    int max_cycles;
    double rtol;
    const double* b_d;        /* GMRES start vector (device)                     */
    const double* v0_d;       /* Arnoldi start vector (device)                   */
    void* ws_d;               /* device workspace of ppa_batch_workspace_bytes  */
    size_t ws_bytes;
} ppa_batch_request;

int ppa_batch_workspace_bytes(int64_t n, int d, int m, int nev, size_t* bytes);
/* Workspace of a request in precision PPA_F64 (as above) or PPA_MIXED, which
 * also holds an FP32 copy of the nnz values and four FP32 n-vectors.
 * PPA_ERR_INVALID for another precision or nnz < 0. */
int ppa_batch_workspace_bytes_ex(int64_t n, int64_t nnz, int d, int m, int nev, int precision,
                                 size_t* bytes);
/* Engine with up to max_slots concurrent solves; all its work goes to `stream`. */
int ppa_batch_create(int max_slots, void* stream, ppa_batch** out);
int ppa_batch_destroy(ppa_batch* b);
/* Admit a request into a free slot (*slot); PPA_ERR_BUSY when none is free. */
int ppa_batch_submit(ppa_batch* b, const ppa_batch_request* rq, int* slot);
/* As ppa_batch_submit, with precision PPA_F64 or PPA_MIXED (mixed precision,
 * section 4's Arnoldi on an FP32 pi(A) until the wanted residuals reach the
 * FP32 floor or stall near it, then the closing FP64 Rayleigh-Ritz pass and,
 * if needed, FP64 cycles from v0_d).  rq->ws_bytes must cover
 * ppa_batch_workspace_bytes_ex for this precision and A's nonzero count
 * (PPA_ERR_WORKSPACE otherwise, before anything is launched); the FP32
 * values are copied from val_d at submit.  PPA_ERR_INVALID for another
 * precision.  Results report fp32_cycles and spmv_passes_f32. */
int ppa_batch_submit_ex(ppa_batch* b, const ppa_batch_request* rq, int precision, int* slot);
/* One launch for all admitted solves, then the host work of the phase ends.
 * finished[0 .. min(*nfinished, cap)) receive slots whose solve ended (their
 * results are ready); *nactive the number of solves that took part.
 * Synchronises the stream. */
int ppa_batch_step(ppa_batch* b, int* finished, int cap, int* nfinished, int* nactive);
/* Results of a finished slot (lam/resid/ritz arrays of capacity nev; X_d is
 * ignored); frees the slot.  Returns the solve's status. */
int ppa_batch_result(ppa_batch* b, int slot, ppa_eigs_result* r);

/* ------------------------------------------------------------------------
 * Host small dense eigensolver used for the projected problems (exported for
 * testing).  a: n x n column-major real matrix (host, not modified).
 * wr, wi: eigenvalues (conjugate pairs adjacent, Im > 0 first).
 * vr, vi: if non-NULL, unit eigenvectors, column j for eigenvalue j.
 * ------------------------------------------------------------------------ */
int ppa_dense_eig(int n, const double* a, double* wr, double* wi, double* vr, double* vi);

/* Modified Leja ordering (section 2, step 1(c)) of a conjugate-closed root set
 * (host arrays, in/out, length n).  Exported for testing. */
int ppa_leja_order(int n, double* re, double* im);

#ifdef __cplusplus
}
#endif

#endif /* PPA_H */
