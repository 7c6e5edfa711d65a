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
    // stream owned by the context on which captured application graphs are
    // replayed, ordered after and before the caller's stream by two events
    hipStream_t graph_stream = nullptr;
    hipEvent_t graph_in = nullptr, graph_out = nullptr;
};

// Application workspace of one operator on one stream (grown on demand).
struct OpWs {
    hipStream_t s;
    double* p;
    size_t bytes;
};
struct ApplyGraph;  // spectral.hip

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
    // how the eigenpairs were obtained (kept by fl_op_save)
    int eig_precision = -1;      // FL_FP64, FL_MIXED, or -1 (installed by the caller)
    int32_t refine_iters = 0;
    double refine_resid = 0.0;
    // application workspaces, one per stream, so calls queued on different
    // streams never share intermediate buffers
    std::vector<OpWs> ws;
    // bandwidth-reducing numbering of the pattern for eigenvalue counting
    // (new index of each old one; device), and the bandwidth under it
    int32_t* inert_pinv = nullptr;
    int64_t inert_bw = -1;
    // half-bandwidth of the pattern in its own numbering (-1: not computed)
    int64_t natural_bw = -1;
    // captured application graphs (fl_apply_graph)
    std::vector<ApplyGraph*> graphs;
    uint64_t graph_clock = 0;
};
// Releases the graphs and workspaces of an operator (device idle).
void fl_op_release_spectral(fl_op* op);

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
hipError_t fl_assemble_csr_launch(hipStream_t s, int elem, const double* xy, const int32_t* conn_sorted,
                                  const int64_t* color_start, int ncolor, const int64_t* dof, const int32_t* rowptr,
                                  const int32_t* colidx, double* kval, double* mval);
hipError_t fl_csr_gather(hipStream_t s, int64_t n, const int32_t* rowptr, const int32_t* colidx, const double* K,
                         const double* M, int64_t ld, double* kval, double* mval);

// apply.hip
hipError_t fl_spmm_csr(hipStream_t s, int64_t n, const int32_t* rowptr, const int32_t* colidx, const double* val,
                       int64_t ncols, const double* X, int64_t ldx, double* Y, int64_t ldy);
hipError_t fl_log_kernel(hipStream_t s, int64_t n, const double* x, double* y);
// Spectral weight families and their parameters for one chunk of at most
// FL_WCHUNK columns, passed to the kernels by value.
enum { FL_SPEC_FRACTIONAL = 0, FL_SPEC_DIFFUSION = 1 };
constexpr int FL_WCHUNK = 32;
struct WeightArgs {
    int kind;
    int count;
    double alpha[FL_WCHUNK];
    double s[FL_WCHUNK];  // diffusion: mu * t
};
hipError_t fl_weights(hipStream_t s, int64_t n, const double* logtheta, const WeightArgs& a, double* W, int64_t ldw);
// U[:, j + i*nf] = V (W[:, i] o C[:, j])   (paired: column b uses W[:, b], C[:, b]).
// forced: launch shape (null: the tuned one, else the built-in default);
// timed: recorded by the kernel timer under "scaled_gemm".
hipError_t fl_scaled_gemm(hipStream_t s, int64_t n, const double* V, int64_t ldv, const double* W, int64_t ldw,
                          const double* C, int64_t ldc, int64_t nf, int64_t na, int paired, double* U,
                          int64_t ldu, const GemmChoice* forced = nullptr, bool timed = true);
// Per-column derivatives of the paired map with respect to the weight
// parameters (chunk a): ga (alpha), gs (mu t; diffusion only, may be null).
hipError_t fl_spec_grad(hipStream_t s, int64_t n, const double* P, int64_t ldp, const double* C, int64_t ldc,
                        const double* W, int64_t ldw, const double* logtheta, const WeightArgs& a, double* ga,
                        double* gs);
// One spectral application queued on stream s with workspace ws (device,
// (2 nf + na) n doubles: G | C | W) and split-k workspace split (null: the
// stream's own).  Queues kernels only: no allocation, no host copy, no
// synchronisation, so it can be captured in a graph.
struct SpecCall {
    int kind;  // FL_SPEC_*
    int64_t nf;
    const double* F;
    int64_t ldf;
    int64_t na;
    const double* alpha;  // host, na
    const double* sprm;   // host, na (diffusion: mu t); null for the fractional kind
    int paired;
    double* U;
    int64_t ldu;
};
hipError_t fl_queue_spectral(const fl_op* op, hipStream_t s, const SpecCall& c, double* ws, const SplitWs* split,
                             bool timed);
size_t fl_spectral_ws_doubles(int64_t n, int64_t nf, int64_t na);
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
// Half-bandwidth max |i - j| of the op's pattern in its own numbering
// (cached in op->natural_bw; inertia.hip).
int fl_pattern_bandwidth(fl_op* op, int64_t* bw);
// Banded mass matrix (q blocks of 128 rows below each diagonal block): the
// factor, L X = B and L^T X = B on the band only (chol.hip).
hipError_t fl_potrf_band(hipStream_t s, int64_t n, int64_t q, double* A, int64_t lda, double* Linv, int64_t* info,
                         double* work);
int64_t fl_band_panel_elems(int64_t n, int64_t q);
hipError_t fl_band_panels(hipStream_t s, int64_t n, int64_t q, const double* L, int64_t ldl, const double* Linv,
                          double* P, int back, GemmProblem* probs);
hipError_t fl_band_solve(hipStream_t s, int64_t n, int64_t q, const double* P, double* B, int64_t ldb, int64_t m,
                         int back, int64_t bwb);
hipError_t fl_trtri_inplace(hipStream_t s, int64_t n, double* L, int64_t ldl, const double* Linv, double* work);
hipError_t fl_symmetrize(hipStream_t s, int64_t n, double* A, int64_t lda);
int fl_sygst_device(fl_ctx* ctx, int64_t n, const double* L, int64_t ldl, const double* Linv, double* K,
                    int64_t ldk, double* work);
// work size (doubles) needed by the TRSMs for an RHS block with `cols` columns / rows
int64_t fl_trsm_work_elems(int64_t n, int64_t other);

// inertia.hip: banded LDL^T of K - sigma M in the operator's bandwidth-reducing
// numbering (new index = inert_pinv[old]).  Bandwidths up to FL_BAND_MAX.
constexpr int FL_BAND_MAX = 511;
int fl_inertia_prepare(fl_op* op);
int64_t fl_band_ldb(int64_t bw);
int64_t fl_band_stride(int64_t n, int64_t bw);
// Factors K - sigma_s M for nshift shifts (sigma_dev: device) into band
// (column layout: L below the diagonal, D on it) and lrow (row layout), each
// nshift * fl_band_stride doubles; neg_dev[s] = negative pivots (or -1).
hipError_t fl_band_factor(hipStream_t s, const fl_op* op, int64_t nshift, const double* sigma_dev, double* band,
                          double* lrow, int64_t* neg_dev);

// sy2sb.hip: number of band-reduction panels for band width b
int64_t fl_sy2sb_panels(int64_t n, int b);
