// extern "C" entry points of libppa.  Each call validates its arguments,
// converts internal exceptions into ppa_status codes and records the message
// for ppa_last_error() (thread-local).
#include <cstdarg>
#include <cstring>
#include <mutex>

#include "ppa_internal.hpp"

#include <cmath>

namespace ppa {

static thread_local std::string g_err;

void fail(int code, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    throw Error(code, buf);
}

void hip_check(hipError_t e, const char* what, const char* file, int line) {
    if (e != hipSuccess)
        fail(PPA_ERR_HIP, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
}

template <class F>
static int guarded(F&& f) {
    try {
        g_err.clear();
        return f();
    } catch (const Error& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return PPA_ERR_INVALID;
    } catch (const std::exception& e) {
        g_err = e.what();
        return PPA_ERR_INVALID;
    }
}

}  // namespace ppa

using namespace ppa;

extern "C" {

int ppa_abi_version(void) { return PPA_ABI_VERSION; }

const char* ppa_last_error(void) { return g_err.c_str(); }

int ppa_matrix_create(int64_t n, const int32_t* rowptr_d, const int32_t* colind_d,
                      const double* val64_d, const float* val32_d, int flags, void* stream,
                      ppa_matrix** out) {
    return guarded([&] {
        PPA_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        PPA_REQUIRE(n >= 1 && n < (int64_t(1) << 31), "n out of range");
        PPA_REQUIRE(rowptr_d && colind_d && val64_d, "rowptr, colind and val64 are required");
        hipStream_t s = (hipStream_t)stream;
        Matrix* A = new Matrix();
        try {
            A->n = n;
            A->rowptr = rowptr_d;
            A->colind = colind_d;
            A->v64 = val64_d;
            A->v32 = val32_d;
            PPA_HIP(hipGetDevice(&A->device));
            matrix_setup(*A, s);
            if (!A->v32 && (flags & PPA_MATRIX_F32) && A->nnz > 0) {
                PPA_HIP(hipMalloc(&A->v32_owned, A->nnz * sizeof(float)));
                launch_cast_f64_f32(A->v64, A->v32_owned, A->nnz, s);
                PPA_HIP(hipStreamSynchronize(s));
                A->v32 = A->v32_owned;
            }
            PPA_REQUIRE(!((flags & PPA_MATRIX_WINDOW_FORCE) && (flags & PPA_MATRIX_RING_FORCE)),
                        "PPA_MATRIX_WINDOW_FORCE and PPA_MATRIX_RING_FORCE exclude each other");
            PPA_REQUIRE(!((flags & PPA_MATRIX_RUNS_FORCE) &&
                          (flags & (PPA_MATRIX_WINDOW_FORCE | PPA_MATRIX_RING_FORCE | PPA_MATRIX_WINDOW_OFF))),
                        "PPA_MATRIX_RUNS_FORCE excludes the other SpMV variant flags");
            const int wmode = (flags & PPA_MATRIX_WINDOW_OFF)     ? -1
                              : (flags & PPA_MATRIX_WINDOW_FORCE) ? 1
                              : (flags & PPA_MATRIX_RING_FORCE)   ? 2
                              : (flags & PPA_MATRIX_RUNS_FORCE)   ? 3
                                                                  : 0;
            matrix_tune(*A, wmode, (flags & PPA_MATRIX_NO_TUNE) == 0, s);
            if (flags & PPA_MATRIX_TWO_STEP) build_two_step(*A, s);
            A->rp_host.clear();
            A->rp_host.shrink_to_fit();
        } catch (...) {
            matrix_release(*A);
            delete A;
            throw;
        }
        *out = reinterpret_cast<ppa_matrix*>(A);
        return PPA_OK;
    });
}

int ppa_matrix_destroy(ppa_matrix* h) {
    return guarded([&] {
        if (!h) return PPA_OK;
        Matrix* A = reinterpret_cast<Matrix*>(h);
        matrix_release(*A);
        delete A;
        return PPA_OK;
    });
}

int ppa_matrix_info(const ppa_matrix* h, int64_t* n, int64_t* nnz, double* norm_inf,
                    int64_t* nblocks) {
    return guarded([&] {
        PPA_REQUIRE(h != nullptr, "matrix is NULL");
        const Matrix* A = reinterpret_cast<const Matrix*>(h);
        if (n) *n = A->n;
        if (nnz) *nnz = A->nnz;
        if (norm_inf) *norm_inf = A->norm_inf;
        if (nblocks) *nblocks = A->nblocks;
        return PPA_OK;
    });
}

int ppa_matrix_spmv_variant(const ppa_matrix* h, int precision, int* windowed) {
    return guarded([&] {
        PPA_REQUIRE(h && windowed, "matrix and windowed are required");
        const Matrix* A = reinterpret_cast<const Matrix*>(h);
        const bool f64 = precision == PPA_F64;
        const Window& W = f64 ? A->win64 : A->win32;
        const Ring& R = f64 ? A->ring64 : A->ring32;
        *windowed = R.on ? 2 : W.on ? 1 : 0;
        return PPA_OK;
    });
}

int ppa_matrix_cache_policy(const ppa_matrix* h, int precision, int* policy) {
    return guarded([&] {
        PPA_REQUIRE(h && policy, "matrix and policy are required");
        PPA_REQUIRE(precision == PPA_F64 || precision == PPA_F32, "precision must be PPA_F64 or PPA_F32");
        const Matrix* A = reinterpret_cast<const Matrix*>(h);
        *policy = precision == PPA_F64 ? A->cp64 : A->cp32;
        return PPA_OK;
    });
}

int ppa_matrix_set_cache_policy(ppa_matrix* h, int precision, int policy) {
    return guarded([&] {
        PPA_REQUIRE(h, "matrix is required");
        PPA_REQUIRE(precision == PPA_F64 || precision == PPA_F32, "precision must be PPA_F64 or PPA_F32");
        PPA_REQUIRE(policy == PPA_CACHE_STREAM || policy == PPA_CACHE_KEEP || policy == PPA_CACHE_KEEP_NTST,
                    "unknown cache policy %d", policy);
        Matrix* A = reinterpret_cast<Matrix*>(h);
        PPA_REQUIRE(precision == PPA_F64 || A->v32, "the matrix has no FP32 values");
        (precision == PPA_F64 ? A->cp64 : A->cp32) = policy;
        return PPA_OK;
    });
}

int ppa_matrix_spmv_blocks(const ppa_matrix* h, int precision, int* nnz_per_block) {
    return guarded([&] {
        PPA_REQUIRE(h && nnz_per_block, "matrix and nnz_per_block are required");
        PPA_REQUIRE(precision == PPA_F64 || precision == PPA_F32, "precision must be PPA_F64 or PPA_F32");
        const Matrix* A = reinterpret_cast<const Matrix*>(h);
        const int b = precision == PPA_F64 ? A->blk64 : A->blk32;
        *nnz_per_block = b == 1 ? SPMV_CHUNK_S : SPMV_CHUNK;
        return PPA_OK;
    });
}

int ppa_matrix_set_spmv_blocks(ppa_matrix* h, int precision, int nnz_per_block) {
    return guarded([&] {
        PPA_REQUIRE(h, "matrix is required");
        PPA_REQUIRE(precision == PPA_F64 || precision == PPA_F32, "precision must be PPA_F64 or PPA_F32");
        PPA_REQUIRE(nnz_per_block == SPMV_CHUNK || nnz_per_block == SPMV_CHUNK_S,
                    "nnz_per_block must be %d or %d", SPMV_CHUNK, SPMV_CHUNK_S);
        Matrix* A = reinterpret_cast<Matrix*>(h);
        PPA_REQUIRE(precision == PPA_F64 || A->v32, "the matrix has no FP32 values");
        (precision == PPA_F64 ? A->blk64 : A->blk32) = nnz_per_block == SPMV_CHUNK_S ? 1 : 0;
        return PPA_OK;
    });
}

int ppa_matrix_spmv_runs(const ppa_matrix* h, int precision, int* on, int64_t* blocks_with_runs) {
    return guarded([&] {
        PPA_REQUIRE(h && on, "matrix and on are required");
        PPA_REQUIRE(precision == PPA_F64 || precision == PPA_F32, "precision must be PPA_F64 or PPA_F32");
        const Matrix* A = reinterpret_cast<const Matrix*>(h);
        const bool f64 = precision == PPA_F64;
        *on = (A->runs.rec && (f64 ? A->runs.on64 : A->runs.on32)) ? 1 : 0;
        if (blocks_with_runs) *blocks_with_runs = A->runs.rec ? (f64 ? A->runs.nwin64 : A->runs.nwin32) : 0;
        return PPA_OK;
    });
}

int ppa_matrix_two_step(const ppa_matrix* h, int precision, int* on, int* bandwidth) {
    return guarded([&] {
        PPA_REQUIRE(h, "matrix is required");
        PPA_REQUIRE(precision == PPA_F64 || precision == PPA_F32, "precision must be PPA_F64 or PPA_F32");
        const Matrix* A = reinterpret_cast<const Matrix*>(h);
        if (on) *on = two_step_on(*A, precision == PPA_F64 ? VecT::F64 : VecT::F32) ? 1 : 0;
        if (bandwidth) *bandwidth = A->two.blk ? A->two.h : -1;
        return PPA_OK;
    });
}

int ppa_matrix_set_two_step(ppa_matrix* h, int precision, int on) {
    return guarded([&] {
        PPA_REQUIRE(h, "matrix is required");
        PPA_REQUIRE(precision == PPA_F64 || precision == PPA_F32, "precision must be PPA_F64 or PPA_F32");
        PPA_REQUIRE(on == 0 || on == 1, "on must be 0 or 1");
        Matrix* A = reinterpret_cast<Matrix*>(h);
        const bool f64 = precision == PPA_F64;
        PPA_REQUIRE(on == 0 || (A->two.blk && (f64 ? A->two.ok64 : A->two.ok32)),
                    "two factors per pass do not fit this matrix and value type");
        (f64 ? A->two.on64 : A->two.on32) = on == 1;
        return PPA_OK;
    });
}

int ppa_matrix_set_spmv_runs(ppa_matrix* h, int precision, int on) {
    return guarded([&] {
        PPA_REQUIRE(h, "matrix is required");
        PPA_REQUIRE(precision == PPA_F64 || precision == PPA_F32, "precision must be PPA_F64 or PPA_F32");
        PPA_REQUIRE(on == 0 || on == 1, "on must be 0 or 1");
        Matrix* A = reinterpret_cast<Matrix*>(h);
        PPA_REQUIRE(precision == PPA_F64 || A->v32, "the matrix has no FP32 values");
        PPA_REQUIRE(on == 0 || A->runs.rec, "no column runs were built for this matrix");
        const bool f64 = precision == PPA_F64;
        (f64 ? A->runs.on64 : A->runs.on32) = on == 1;
        if (on) (f64 ? A->blk64 : A->blk32) = 0;
        return PPA_OK;
    });
}

static std::vector<cplx> read_roots(int deg, const double* re, const double* im) {
    PPA_REQUIRE(deg >= 1 && re, "polynomial needs deg >= 1 roots");
    std::vector<cplx> r(deg);
    for (int i = 0; i < deg; ++i) {
        r[i] = cplx(re[i], im ? im[i] : 0.0);
        PPA_REQUIRE(std::isfinite(re[i]) && std::isfinite(r[i].imag()), "root %d is not finite", i);
        PPA_REQUIRE(r[i] != cplx(0.0, 0.0), "root %d is zero", i);
    }
    for (int i = 0; i < deg;) {
        if (r[i].imag() != 0.0) {
            PPA_REQUIRE(r[i].imag() > 0.0 && i + 1 < deg && r[i + 1] == std::conj(r[i]),
                        "complex root %d must have Im > 0 and be followed by its conjugate", i);
            i += 2;
        } else {
            i += 1;
        }
    }
    return r;
}

int ppa_poly_from_roots(int deg, const double* re, const double* im, int d1, const double* re1,
                        const double* im1, ppa_poly** out) {
    return guarded([&] {
        PPA_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        Poly* p = new Poly();
        try {
            p->roots = read_roots(deg, re, im);
            if (d1 > 0) p->roots1 = read_roots(d1, re1, im1);
        } catch (...) {
            delete p;
            throw;
        }
        *out = reinterpret_cast<ppa_poly*>(p);
        return PPA_OK;
    });
}

int ppa_poly_destroy(ppa_poly* p) {
    delete reinterpret_cast<Poly*>(p);
    return PPA_OK;
}

int ppa_poly_degree(const ppa_poly* h, int* deg, int* d1) {
    return guarded([&] {
        PPA_REQUIRE(h != nullptr, "poly is NULL");
        const Poly* p = reinterpret_cast<const Poly*>(h);
        if (deg) *deg = (int)p->roots.size();
        if (d1) *d1 = (int)p->roots1.size();
        return PPA_OK;
    });
}

int ppa_poly_roots(const ppa_poly* h, int level, double* re, double* im, int cap, int* count) {
    return guarded([&] {
        PPA_REQUIRE(h != nullptr, "poly is NULL");
        const Poly* p = reinterpret_cast<const Poly*>(h);
        PPA_REQUIRE(level == 1 || level == 2, "level must be 1 or 2");
        const std::vector<cplx>& r = level == 2 ? p->roots : p->roots1;
        PPA_REQUIRE((int)r.size() <= cap, "capacity %d below the root count %zu", cap, r.size());
        for (size_t i = 0; i < r.size(); ++i) {
            if (re) re[i] = r[i].real();
            if (im) im[i] = r[i].imag();
        }
        if (count) *count = (int)r.size();
        return PPA_OK;
    });
}

int ppa_poly_log10_pof(const ppa_poly* h, int level, double* out, int cap, int* count) {
    return guarded([&] {
        PPA_REQUIRE(h != nullptr && out != nullptr, "poly and out are required");
        PPA_REQUIRE(level == 1 || level == 2, "level must be 1 or 2");
        const Poly* p = reinterpret_cast<const Poly*>(h);
        const std::vector<cplx>& r = level == 2 ? p->roots : p->roots1;
        PPA_REQUIRE((int)r.size() <= cap, "capacity %d below the root count %zu", cap, r.size());
        const std::vector<double> lp = log10_pof(r);
        for (size_t i = 0; i < lp.size(); ++i) out[i] = lp[i];
        if (count) *count = (int)lp.size();
        return PPA_OK;
    });
}

int ppa_poly_stabilize(const ppa_poly* h, int level, ppa_poly** out, int* added) {
    return guarded([&] {
        PPA_REQUIRE(h != nullptr && out != nullptr, "poly and out are required");
        PPA_REQUIRE(level == 1 || level == 2, "level must be 1 or 2");
        *out = nullptr;
        const Poly* p = reinterpret_cast<const Poly*>(h);
        PPA_REQUIRE(level == 2 || p->is_double(), "level 1 needs a double polynomial");
        Poly* q = new Poly(*p);
        int n_added = 0;
        if (level == 2)
            q->roots = add_stability_roots(p->roots, &n_added);
        else
            q->roots1 = add_stability_roots(p->roots1, &n_added);
        if (added) *added = n_added;
        *out = reinterpret_cast<ppa_poly*>(q);
        return PPA_OK;
    });
}

int ppa_poly_build_workspace_bytes(const ppa_matrix* h, int d, int double_poly, size_t* bytes) {
    return guarded([&] {
        PPA_REQUIRE(h && bytes, "matrix and bytes are required");
        PPA_REQUIRE(d >= 1, "degree must be >= 1");
        *bytes = poly_build_ws(reinterpret_cast<const Matrix*>(h)->n, d, double_poly != 0);
        return PPA_OK;
    });
}

int ppa_poly_build(const ppa_matrix* h, int d, const double* b_d, void* ws_d, size_t ws_bytes,
                   void* stream, ppa_poly** out) {
    return guarded([&] {
        PPA_REQUIRE(h && b_d && out, "matrix, b and out are required");
        *out = nullptr;
        Poly* p = new Poly();
        int st;
        try {
            st = poly_build(*reinterpret_cast<const Matrix*>(h), d, 0, b_d, ws_d, ws_bytes,
                            (hipStream_t)stream, *p);
        } catch (...) {
            delete p;
            throw;
        }
        *out = reinterpret_cast<ppa_poly*>(p);
        return st;
    });
}

int ppa_poly_build_double(const ppa_matrix* h, int d1, int d2, const double* b_d, void* ws_d,
                          size_t ws_bytes, void* stream, ppa_poly** out) {
    return guarded([&] {
        PPA_REQUIRE(h && b_d && out, "matrix, b and out are required");
        PPA_REQUIRE(d2 >= 1, "d2 must be >= 1");
        *out = nullptr;
        Poly* p = new Poly();
        int st;
        try {
            st = poly_build(*reinterpret_cast<const Matrix*>(h), d1, d2, b_d, ws_d, ws_bytes,
                            (hipStream_t)stream, *p);
        } catch (...) {
            delete p;
            throw;
        }
        *out = reinterpret_cast<ppa_poly*>(p);
        return st;
    });
}

int ppa_poly_shift(const ppa_poly* h, double* shift) {
    return guarded([&] {
        PPA_REQUIRE(h && shift, "poly and shift are required");
        *shift = reinterpret_cast<const Poly*>(h)->shift;
        return PPA_OK;
    });
}

int ppa_poly_set_shift(ppa_poly* h, double shift) {
    return guarded([&] {
        PPA_REQUIRE(h != nullptr, "poly is NULL");
        PPA_REQUIRE(std::isfinite(shift), "shift must be finite");
        reinterpret_cast<Poly*>(h)->shift = shift;
        return PPA_OK;
    });
}

int ppa_poly_build_ex_workspace_bytes(const ppa_matrix* h, const ppa_poly_build_opts* o,
                                      int two_start, size_t* bytes) {
    return guarded([&] {
        PPA_REQUIRE(h && o && bytes, "matrix, options and bytes are required");
        PPA_REQUIRE(o->d >= 1, "degree must be >= 1");
        *bytes = poly_build_ex_ws(*reinterpret_cast<const Matrix*>(h), *o, two_start != 0);
        return PPA_OK;
    });
}

int ppa_poly_build_ex(const ppa_matrix* h, const ppa_poly_build_opts* o, const double* b_d,
                      const double* b2_d, void* ws_d, size_t ws_bytes, void* stream,
                      ppa_poly** out, ppa_poly_build_info* info) {
    return guarded([&] {
        PPA_REQUIRE(h && o && b_d && out, "matrix, options, b and out are required");
        *out = nullptr;
        PPA_REQUIRE(ws_d != nullptr, "workspace is required");
        Poly* p = new Poly();
        ppa_poly_build_info inf{};
        int st = PPA_OK;
        try {
            st = poly_build_ex(*reinterpret_cast<const Matrix*>(h), *o, b_d, b2_d, ws_d, ws_bytes,
                               (hipStream_t)stream, *p, inf);
        } catch (...) {
            delete p;
            throw;
        }
        if (info) *info = inf;
        *out = reinterpret_cast<ppa_poly*>(p);
        return st;
    });
}

int ppa_poly_apply_workspace_bytes(const ppa_matrix* h, const ppa_poly* ph, int precision,
                                   size_t* bytes) {
    return guarded([&] {
        PPA_REQUIRE(h && ph && bytes, "matrix, poly and bytes are required");
        PPA_REQUIRE(precision == PPA_F64 || precision == PPA_F32, "precision must be F64 or F32");
        Carver c(nullptr, 0);
        ApplyWs aw;
        carve_apply(c, reinterpret_cast<const Matrix*>(h)->n, *reinterpret_cast<const Poly*>(ph),
                    precision == PPA_F64 ? VecT::F64 : VecT::F32, aw);
        *bytes = c.bytes();
        return PPA_OK;
    });
}

int ppa_poly_apply(const ppa_matrix* h, const ppa_poly* ph, int precision, const void* v_d,
                   void* y_d, void* ws_d, size_t ws_bytes, void* stream) {
    return guarded([&] {
        PPA_REQUIRE(h && ph && v_d && y_d, "matrix, poly, v and y are required");
        PPA_REQUIRE(v_d != y_d, "v and y must not alias");
        PPA_REQUIRE(precision == PPA_F64 || precision == PPA_F32, "precision must be F64 or F32");
        const Matrix& A = *reinterpret_cast<const Matrix*>(h);
        const Poly& p = *reinterpret_cast<const Poly*>(ph);
        const VecT t = precision == PPA_F64 ? VecT::F64 : VecT::F32;
        Carver c(ws_d, ws_bytes);
        ApplyWs aw;
        carve_apply(c, A.n, p, t, aw);
        PPA_REQUIRE(ws_d != nullptr, "workspace is required");
        c.check();
        apply_poly(A, p, t, v_d, t, y_d, t, aw, (hipStream_t)stream);
        return PPA_OK;
    });
}

int ppa_poly_apply_bytes(const ppa_matrix* h, const ppa_poly* ph, int precision, double* bytes) {
    return guarded([&] {
        PPA_REQUIRE(h && ph && bytes, "matrix, poly and bytes are required");
        PPA_REQUIRE(precision == PPA_F64 || precision == PPA_F32, "precision must be F64 or F32");
        const Matrix& A = *reinterpret_cast<const Matrix*>(h);
        *bytes = (double)apply_poly_bytes(A, *reinterpret_cast<const Poly*>(ph),
                                          precision == PPA_F64 ? VecT::F64 : VecT::F32);
        return PPA_OK;
    });
}

int ppa_fused_spmv(const ppa_matrix* h, int in_f32, int out_f32, double alpha, const void* x_d,
                   double beta, const void* u_d, double gamma, const void* z_d, double delta,
                   const void* z2_d, void* out_d, void* stream) {
    return guarded([&] {
        PPA_REQUIRE(h != nullptr, "matrix is NULL");
        launch_fused_spmv(*reinterpret_cast<const Matrix*>(h), in_f32 ? VecT::F32 : VecT::F64,
                          out_f32 ? VecT::F32 : VecT::F64, alpha, x_d, beta, u_d, gamma, z_d,
                          delta, z2_d, out_d, (hipStream_t)stream);
        return PPA_OK;
    });
}

int ppa_cgs2_workspace_bytes(int64_t n, int j, size_t* bytes) {
    return guarded([&] {
        PPA_REQUIRE(bytes && n >= 1 && j >= 1, "bad arguments");
        Carver c(nullptr, 0);
        Cgs2Ws w;
        carve_cgs2(c, n, w);
        c.take<double>(CGS_JMAX_ALL);
        *bytes = c.bytes();
        return PPA_OK;
    });
}

int ppa_cgs2(int64_t n, int j, const double* V_d, int64_t ldv, double* w_d, double* h,
             double* w0norm, void* ws_d, size_t ws_bytes, void* stream) {
    return guarded([&] {
        PPA_REQUIRE(V_d && w_d && h && ws_d, "V, w, h and workspace are required");
        PPA_REQUIRE(n >= 1 && j >= 1 && j < CGS_JMAX_ALL - 1 && ldv >= n, "bad sizes");
        Carver c(ws_d, ws_bytes);
        Cgs2Ws w;
        carve_cgs2(c, n, w);
        double* Hcol = c.take<double>(CGS_JMAX_ALL);
        c.check();
        hipStream_t s = (hipStream_t)stream;
        launch_cgs2(n, j, V_d, ldv, w_d, w_d, Hcol, nullptr, 0.0, w, s);
        PPA_HIP(hipMemcpyAsync(h, Hcol, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
        double sc[3];
        PPA_HIP(hipMemcpyAsync(sc, w.scal, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        PPA_HIP(hipStreamSynchronize(s));
        if (w0norm) *w0norm = std::sqrt(sc[0]);
        return PPA_OK;
    });
}

int ppa_gemm_workspace_bytes(int kin, int kout, size_t* bytes) {
    return guarded([&] {
        PPA_REQUIRE(bytes && kin >= 1 && kout >= 1, "bad arguments");
        *bytes = ((size_t)kin * kout * sizeof(double) + 255) & ~size_t(255);
        return PPA_OK;
    });
}

int ppa_gemm_tall(int64_t n, int kin, int kout, const double* V_d, int64_t ldv, const double* Q,
                  double* C_d, int64_t ldc, void* ws_d, size_t ws_bytes, void* stream) {
    return guarded([&] {
        PPA_REQUIRE(V_d && Q && C_d && ws_d, "V, Q, C and workspace are required");
        PPA_REQUIRE(ldv >= n && ldc >= n, "leading dimensions must be >= n");
        PPA_REQUIRE(ws_bytes >= (size_t)kin * kout * sizeof(double), "workspace too small");
        hipStream_t s = (hipStream_t)stream;
        PPA_HIP(hipMemcpyAsync(ws_d, Q, (size_t)kin * kout * sizeof(double), hipMemcpyHostToDevice, s));
        launch_gemm_tall(n, kin, kout, V_d, ldv, (const double*)ws_d, C_d, ldc, s);
        return PPA_OK;
    });
}

int ppa_eigs_workspace_bytes(const ppa_matrix* h, const ppa_poly* ph, const ppa_eigs_opts* o,
                             size_t* bytes) {
    return guarded([&] {
        PPA_REQUIRE(h && o && bytes, "matrix, opts and bytes are required");
        *bytes = eigs_ws(*reinterpret_cast<const Matrix*>(h), reinterpret_cast<const Poly*>(ph), *o);
        return PPA_OK;
    });
}

int ppa_eigs(const ppa_matrix* h, const ppa_poly* ph, const ppa_eigs_opts* o, const double* v0_d,
             void* ws_d, size_t ws_bytes, void* stream, ppa_eigs_result* r) {
    return guarded([&] {
        PPA_REQUIRE(h && o && v0_d && r && ws_d, "matrix, opts, v0, result and workspace are required");
        return eigs(*reinterpret_cast<const Matrix*>(h), reinterpret_cast<const Poly*>(ph), *o, v0_d,
                    ws_d, ws_bytes, (hipStream_t)stream, *r);
    });
}

int ppa_batch_workspace_bytes(int64_t n, int d, int m, int nev, size_t* bytes) {
    return guarded([&] {
        PPA_REQUIRE(bytes && n >= 1 && d >= 1 && m >= 2 && nev >= 1, "bad arguments");
        *bytes = batch_ws_bytes(n, d, m, nev);
        return PPA_OK;
    });
}

int ppa_batch_workspace_bytes_ex(int64_t n, int64_t nnz, int d, int m, int nev, int precision,
                                 size_t* bytes) {
    return guarded([&] {
        PPA_REQUIRE(bytes && n >= 1 && d >= 1 && m >= 2 && nev >= 1 && nnz >= 0, "bad arguments");
        PPA_REQUIRE(precision == PPA_F64 || precision == PPA_MIXED, "precision must be F64 or MIXED");
        *bytes = batch_ws_bytes(n, d, m, nev, nnz, precision);
        return PPA_OK;
    });
}

int ppa_batch_create(int max_slots, void* stream, ppa_batch** out) {
    return guarded([&] {
        PPA_REQUIRE(out != nullptr, "out is NULL");
        *out = reinterpret_cast<ppa_batch*>(batch_create(max_slots, (hipStream_t)stream));
        return PPA_OK;
    });
}

int ppa_batch_destroy(ppa_batch* b) {
    return guarded([&] {
        batch_destroy(reinterpret_cast<Batch*>(b));
        return PPA_OK;
    });
}

int ppa_batch_submit(ppa_batch* b, const ppa_batch_request* rq, int* slot) {
    return guarded([&] {
        PPA_REQUIRE(b && rq && slot, "batch, request and slot are required");
        return batch_submit(*reinterpret_cast<Batch*>(b), *rq, slot);
    });
}

int ppa_batch_submit_ex(ppa_batch* b, const ppa_batch_request* rq, int precision, int* slot) {
    return guarded([&] {
        PPA_REQUIRE(b && rq && slot, "batch, request and slot are required");
        return batch_submit(*reinterpret_cast<Batch*>(b), *rq, slot, precision);
    });
}

int ppa_batch_step(ppa_batch* b, int* finished, int cap, int* nfinished, int* nactive) {
    return guarded([&] {
        PPA_REQUIRE(b && nfinished, "batch and nfinished are required");
        return batch_step(*reinterpret_cast<Batch*>(b), finished, cap, nfinished, nactive);
    });
}

int ppa_batch_result(ppa_batch* b, int slot, ppa_eigs_result* r) {
    return guarded([&] {
        PPA_REQUIRE(b && r, "batch and result are required");
        return batch_result(*reinterpret_cast<Batch*>(b), slot, *r);
    });
}

int ppa_dense_eig(int n, const double* a, double* wr, double* wi, double* vr, double* vi) {
    return guarded([&] {
        PPA_REQUIRE(n >= 1 && a && wr && wi, "bad arguments");
        std::vector<cplx> w, V;
        dense_eig(n, a, w, (vr || vi) ? &V : nullptr);
        for (int i = 0; i < n; ++i) {
            wr[i] = w[i].real();
            wi[i] = w[i].imag();
        }
        if (vr || vi)
            for (size_t i = 0; i < (size_t)n * n; ++i) {
                if (vr) vr[i] = V[i].real();
                if (vi) vi[i] = V[i].imag();
            }
        return PPA_OK;
    });
}

int ppa_leja_order(int n, double* re, double* im) {
    return guarded([&] {
        PPA_REQUIRE(n >= 0 && (n == 0 || (re && im)), "bad arguments");
        std::vector<cplx> t(n);
        for (int i = 0; i < n; ++i) t[i] = cplx(re[i], im[i]);
        const std::vector<cplx> o = leja_order(t);
        for (int i = 0; i < n; ++i) {
            re[i] = o[i].real();
            im[i] = o[i].imag();
        }
        return PPA_OK;
    });
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free apply
// The polynomial chain's temporaries of ppa_poly_apply_noalloc live in one
// file-scope device array (each device that runs the call holds its own copy
// until the process ends).  Host code never passes the array's name to a
// kernel or a copy: it is only a host-side stand-in.  The device address is
// looked up once per device, with that device current, and cached.
namespace {

static __device__ __align__(256) unsigned char scratch[PPA_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* scratch_on_current_device() {
    int dev = 0;
    PPA_HIP(hipGetDevice(&dev));
    PPA_REQUIRE(dev >= 0 && dev < kMaxDevices, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        PPA_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        PPA_REQUIRE(ptr != nullptr, "no device address for the static scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" int ppa_poly_apply_noalloc(const ppa_matrix* h, const ppa_poly* ph, int precision,
                                      const void* v_d, void* y_d, void* stream) {
    return guarded([&] {
        PPA_REQUIRE(h && ph && v_d && y_d, "matrix, poly, v and y are required");
        PPA_REQUIRE(v_d != y_d, "v and y must not alias");
        PPA_REQUIRE(precision == PPA_F64 || precision == PPA_F32, "precision must be F64 or F32");
        const Matrix& A = *reinterpret_cast<const Matrix*>(h);
        const Poly& p = *reinterpret_cast<const Poly*>(ph);
        const VecT t = precision == PPA_F64 ? VecT::F64 : VecT::F32;
        // size check first, on the host: nothing is launched for a request
        // that does not fit
        {
            Carver dry(nullptr, 0);
            ApplyWs probe;
            carve_apply(dry, A.n, p, t, probe);
            if (dry.bytes() > (size_t)PPA_NOALLOC_SCRATCH_BYTES)
                fail(PPA_ERR_WORKSPACE,
                     "ppa_poly_apply_noalloc: needs %zu bytes of scratch, the static array holds %zu "
                     "(use ppa_poly_apply with a workspace)",
                     dry.bytes(), (size_t)PPA_NOALLOC_SCRATCH_BYTES);
        }
        int dev = 0;
        PPA_HIP(hipGetDevice(&dev));
        PPA_REQUIRE(dev == A.device, "the current device (%d) is not the matrix's (%d)", dev, A.device);
        void* base = scratch_on_current_device();
        Carver c(base, PPA_NOALLOC_SCRATCH_BYTES);
        ApplyWs aw;
        carve_apply(c, A.n, p, t, aw);
        c.check();
        // every temporary of the chain is written by a pass before any pass
        // reads it, so the previous call's contents need no clearing
        apply_poly(A, p, t, v_d, t, y_d, t, aw, (hipStream_t)stream);
        return PPA_OK;
    });
}
