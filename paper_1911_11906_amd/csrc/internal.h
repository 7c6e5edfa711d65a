// Internal state and launchers of the fraclap library.
#pragma once
#include <algorithm>
#include <string>
#include <vector>
#include "common.h"
#include "../../include/fraclap.h"

struct fl_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // band of the bulge chase in uncached memory, grown on demand and never
    // freed (see band_buffer in eig.hip)
    void* band_uc = nullptr;
    size_t band_uc_bytes = 0;
};

struct fl_op {
    fl_ctx* ctx = nullptr;
    int device = 0;          // copy of ctx->device: destroy must not depend on the context
    int64_t n = 0;
    int64_t ld = 0;          // leading dimension of every n x n device array of the op
    double* K = nullptr;     // dense, device
    double* M = nullptr;     // dense, device
    // CSR pattern shared by K and M (rows sorted), device
    int64_t nnz = 0;
    int32_t* rowptr = nullptr;
    int32_t* colidx = nullptr;
    double* kval = nullptr;
    double* mval = nullptr;
    // eigenpairs
    int has_eig = 0;
    double* theta = nullptr;     // n
    double* logtheta = nullptr;  // n
    double* V = nullptr;         // n x n, ld
    // apply workspace (grown on demand)
    double* ws = nullptr;
    size_t ws_bytes = 0;
};

// Optional per-kernel timing (ktimer.hip): events around one launch when
// timing is enabled; a no-op otherwise.
struct KScope {
    KScope(const char* name, hipStream_t s);
    ~KScope();
    KScope(const KScope&) = delete;
    KScope& operator=(const KScope&) = delete;

   private:
    const char* name_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
    bool on_ = false;
};

// status helpers ------------------------------------------------------------
int fl_fail(fl_ctx* ctx, int code, const std::string& msg);
#define FL_HIP(ctx, expr)                                                                     \
    do {                                                                                      \
        hipError_t e__ = (expr);                                                              \
        if (e__ != hipSuccess)                                                                \
            return fl_fail((ctx), FL_EHIP, std::string(#expr ": ") + hipGetErrorString(e__)); \
    } while (0)

// device buffer that frees itself
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    hipError_t alloc(size_t b) {
        release();
        bytes = b;
        return hipMalloc(&p, b > 0 ? b : 16);
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// assemble.hip
hipError_t fl_assemble_launch(hipStream_t s, int elem, const double* xy, const int32_t* conn_sorted,
                              const int64_t* color_start, int ncolor, const int64_t* dof_of_node, int64_t n,
                              int64_t ld, double* K, double* M);
hipError_t fl_csr_gather(hipStream_t s, int64_t n, const int32_t* rowptr, const int32_t* colidx, const double* K,
                         const double* M, int64_t ld, double* kval, double* mval);

// apply.hip
hipError_t fl_spmm_csr(hipStream_t s, int64_t n, const int32_t* rowptr, const int32_t* colidx, const double* val,
                       int64_t ncols, const double* X, int64_t ldx, double* Y, int64_t ldy);
hipError_t fl_log_kernel(hipStream_t s, int64_t n, const double* x, double* y);
hipError_t fl_weights(hipStream_t s, int64_t n, const double* logtheta, int64_t na, const double* alpha_dev,
                      double* W, int64_t ldw);
// U[:, j + i*nf] = V (W[:, i] o C[:, j])   (paired: column b uses W[:, b], C[:, b])
hipError_t fl_scaled_gemm(hipStream_t s, int64_t n, const double* V, int64_t ldv, const double* W, int64_t ldw,
                          const double* C, int64_t ldc, int64_t nf, int64_t na, int paired, double* U,
                          int64_t ldu);
hipError_t fl_galpha(hipStream_t s, int64_t n, int64_t nb, const double* P, int64_t ldp, const double* C,
                     int64_t ldc, const double* W, int64_t ldw, const double* logtheta, double* galpha_dev);
hipError_t fl_check_finite(hipStream_t s, int64_t m, int64_t n, const double* A, int64_t lda, int* flag_dev);

// chol.hip
// Blocked recursive Cholesky; writes 1-based failing pivot (or 0) to info_dev.
// Linv: workspace of n_leaf blocks of 128 x 128 (inverses of the diagonal blocks).
int64_t fl_potrf_linv_elems(int64_t n);
hipError_t fl_potrf(hipStream_t s, int64_t n, double* A, int64_t lda, double* Linv, int64_t* info_dev,
                    double* work);
// X L^T = B (B overwritten by X), L lower from fl_potrf with its Linv.
hipError_t fl_trsm_rlt(hipStream_t s, int64_t m, int64_t k, const double* L, int64_t ldl, const double* Linv,
                       double* B, int64_t ldb, double* work);
// L X = B
hipError_t fl_trsm_lln(hipStream_t s, int64_t k, int64_t m, const double* L, int64_t ldl, const double* Linv,
                       double* B, int64_t ldb, double* work);
// L^T X = B
hipError_t fl_trsm_llt(hipStream_t s, int64_t k, int64_t m, const double* L, int64_t ldl, const double* Linv,
                       double* B, int64_t ldb, double* work);
hipError_t fl_trtri_leaves(hipStream_t s, int64_t n, const double* L, int64_t ldl, double* Linv);
hipError_t fl_trtri_inplace(hipStream_t s, int64_t n, double* L, int64_t ldl, const double* Linv, double* work);
hipError_t fl_symmetrize(hipStream_t s, int64_t n, double* A, int64_t lda);
int fl_sygst_device(fl_ctx* ctx, int64_t n, const double* L, int64_t ldl, const double* Linv, double* K,
                    int64_t ldk, double* work);
// work size (doubles) needed by the TRSMs for an RHS block with `cols` columns / rows
int64_t fl_trsm_work_elems(int64_t n, int64_t other);

// sy2sb.hip: number of band-reduction panels for band width b
int64_t fl_sy2sb_panels(int64_t n, int b);
