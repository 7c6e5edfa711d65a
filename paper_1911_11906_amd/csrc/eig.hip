// The full-spectrum generalized eigensolve K phi = theta M phi (eq.
// discrete_laplace) with M-orthonormal eigenvectors (Section
// "Post-processing"), as a dense FP64 pipeline on one GPU:
//   M = L L^T;  C = L^-1 K L^-T;  C -> band -> tridiagonal T (two stages);
//   T = Z_T diag(theta) Z_T^T (divide and conquer);  Z = Q1 Q2 Z_T;  V = L^-T Z.
// V^T M V = Z^T L^-1 L L^T L^-T Z = Z^T Z = I.
#include <algorithm>
#include <cmath>
#include <vector>
#include "internal.h"

// sy2sb.hip
hipError_t fl_sy2sb(hipStream_t s, int64_t n, int b, double* A, int64_t lda, double* V1, int64_t ldv, double* T1,
                    double* tau1, double* work, double* part, unsigned* cnt, int* abort);
int64_t fl_sy2sb_work_elems(int64_t n, int b);
int64_t fl_sy2sb_part_elems(int64_t n);
hipError_t fl_extract_band(hipStream_t s, int64_t n, int b, const double* A, int64_t lda, double* AB, int64_t ldab);
// sb2st.hip
int64_t fl_sb2st_maxt(int64_t n, int b);
hipError_t fl_sb2st(hipStream_t s, int64_t n, int b, double* AB, int64_t ldab, double* d, double* e, double* V2,
                    double* tau2, int* prog, int grid, int* abort);
// backtrans.hip
int64_t fl_q2_t_elems(int64_t n, int b, int64_t maxt);
int64_t fl_q1_work_elems(int64_t n, int b, int64_t ncols);
hipError_t fl_q2_apply(hipStream_t s, int64_t n, int b, const double* V2, const double* tau2, int64_t maxt, double* T2,
                       double* Z, int64_t ldz, int64_t ncols);
hipError_t fl_q1_apply(hipStream_t s, int64_t n, int b, const double* V1, int64_t ldv, const double* T1, double* Z,
                       int64_t ldz, int64_t ncols, double* work);
hipError_t fl_ssy2sb(hipStream_t s, int64_t n, int b, float* A, int64_t lda, float* V1, int64_t ldv, float* T1,
                     float* tau1, float* work, float* part, unsigned* cnt, int* abort);
hipError_t fl_extract_band_f(hipStream_t s, int64_t n, int b, const float* A, int64_t lda, double* AB, int64_t ldab);
hipError_t fl_q2_apply_f(hipStream_t s, int64_t n, int b, const double* V2, const double* tau2, int64_t maxt,
                         float* work, float* Z, int64_t ldz, int64_t ncols);
hipError_t fl_q1_apply_f(hipStream_t s, int64_t n, int b, const float* V1, int64_t ldv, const float* T1, float* Z,
                         int64_t ldz, int64_t ncols, float* work);
// stedc.hip
int fl_stedc_device(fl_ctx* ctx, int64_t n, double* d, const double* e, double* Zout, int64_t ldz, int leaf);
// refine.hip
int fl_refine_device(fl_ctx* ctx, fl_op* op, double* theta, double* X, int64_t ldx, int max_iters, double tol,
                     fl_eig_info* info, int64_t partial);
int fl_rayleigh_device(fl_ctx* ctx, fl_op* op, double* theta, double* X, int64_t ldx);

namespace {

struct StageTimer {
    hipStream_t s;
    std::vector<hipEvent_t> ev;
    std::vector<int> stage;
    explicit StageTimer(hipStream_t st) : s(st) {}
    ~StageTimer() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    hipError_t mark(int st) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        ev.push_back(e);
        stage.push_back(st);
        return hipEventRecord(e, s);
    }
    // stage_ms[stage[k]] += time between mark k and k+1
    void collect(fl_eig_info* info) {
        if (!info) return;
        for (size_t k = 0; k + 1 < ev.size(); ++k) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) == hipSuccess && stage[k] >= 0) info->stage_ms[stage[k]] += ms;
        }
        float tot = 0.f;
        if (ev.size() >= 2 && hipEventElapsedTime(&tot, ev.front(), ev.back()) == hipSuccess) info->total_ms = tot;
    }
};

int clamp_band(int64_t n, int band) {
    int b = band > 0 ? band : 64;
    b = std::max(2, std::min(b, 64));
    return b;
}

// Band of the bulge chase.  Every task hands its blocks to a sweep on another
// XCD, so the L2 keeps nothing reusable of it; in uncached memory the
// agent-scope release and acquire of each task find no band lines to write
// back or drop.  Uncached memory is not freed while the process runs (memory
// allocated after such a free has been seen to hold wrong values), so the
// context keeps one buffer, replaced by a larger one when needed (the old
// one stays allocated).  Falls back to ordinary memory (returns null).
double* band_buffer(fl_ctx* ctx, size_t bytes) {
    if (ctx->band_uc_bytes < bytes) {
        void* p = nullptr;
        if (hipExtMallocWithFlags(&p, bytes, hipDeviceMallocUncached) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        ctx->band_uc = p;
        ctx->band_uc_bytes = bytes;
    }
    return static_cast<double*>(ctx->band_uc);
}

int grid_for_sb2st(int64_t n, int b) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    }
    // sweeps start about two tasks apart, so about n / 2b of them are active
    int64_t useful = n / (2 * (int64_t)b) + 2;
    return (int)std::max<int64_t>(1, std::min<int64_t>(useful, cus));
}

}  // namespace

// Two-stage tridiagonalisation + D&C + back-transforms of the symmetric A
// (full storage, destroyed).  w (n) ascending, Z (n x n, ld ldz).
int fl_syevd_device(fl_ctx* ctx, int64_t n, double* A, int64_t lda, int band, double* w, double* Z, int64_t ldz,
                    fl_eig_info* info, int leaf, StageTimer* tm_ext = nullptr);

int fl_syevd_device(fl_ctx* ctx, int64_t n, double* A, int64_t lda, int band, double* w, double* Z, int64_t ldz,
                    fl_eig_info* info, int leaf, StageTimer* tm) {
    hipStream_t s = ctx->stream;
    const int b = clamp_band(n, band);
    const int64_t ldab = 2 * b + 1;
    const int64_t np = std::max<int64_t>(1, fl_sy2sb_panels(n, b));
    const int64_t maxt = fl_sb2st_maxt(n, b);
    const int64_t nsw = std::max<int64_t>(1, n - 2);
    DevBuf bAB, bV1, bT1, btau1, bwork, bpart, bcnt, bV2, btau2, bprog, bT2, be;
    double* ABp = band_buffer(ctx, sizeof(double) * ldab * n);
    if (!ABp) {
        FL_HIP(ctx, bAB.alloc(sizeof(double) * ldab * n));
        ABp = bAB.as<double>();
    }
    FL_HIP(ctx, bV1.alloc(sizeof(double) * (size_t)n * n));
    FL_HIP(ctx, hipMemsetAsync(bV1.p, 0, sizeof(double) * (size_t)n * n, s));  // Q1 reads above each panel
    FL_HIP(ctx, bT1.alloc(sizeof(double) * np * b * b));
    FL_HIP(ctx, btau1.alloc(sizeof(double) * (n + b)));
    FL_HIP(ctx, bwork.alloc(sizeof(double) * std::max<int64_t>(fl_sy2sb_work_elems(n, b), fl_q1_work_elems(n, b, n))));
    FL_HIP(ctx, bpart.alloc(sizeof(double) * fl_sy2sb_part_elems(n)));
    FL_HIP(ctx, bcnt.alloc(sizeof(unsigned) * np));
    FL_HIP(ctx, bV2.alloc(sizeof(double) * nsw * maxt * b));
    FL_HIP(ctx, btau2.alloc(sizeof(double) * nsw * maxt));
    FL_HIP(ctx, bprog.alloc(sizeof(int) * (2 * n + 2)));
    FL_HIP(ctx, be.alloc(sizeof(double) * (n + 1)));
    double* e = be.as<double>();
    int* abort_flag = bprog.as<int>() + 2 * n + 1;
    FL_HIP(ctx, hipMemsetAsync(abort_flag, 0, sizeof(int), s));

    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_SY2SB));
    FL_HIP(ctx, fl_sy2sb(s, n, b, A, lda, bV1.as<double>(), n, bT1.as<double>(), btau1.as<double>(),
                         bwork.as<double>(), bpart.as<double>(), bcnt.as<unsigned>(), abort_flag));
    FL_HIP(ctx, fl_extract_band(s, n, b, A, lda, ABp, ldab));
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_SB2ST));
    FL_HIP(ctx, fl_sb2st(s, n, b, ABp, ldab, w, e, bV2.as<double>(), btau2.as<double>(), bprog.as<int>(),
                         grid_for_sb2st(n, b), abort_flag));
    {
        int ab = 0;
        FL_HIP(ctx, hipMemcpyAsync(&ab, abort_flag, sizeof(int), hipMemcpyDeviceToHost, s));
        FL_HIP(ctx, hipStreamSynchronize(s));
        if (ab) {
            if (info) info->index = FL_STAGE_SB2ST;
            return fl_fail(ctx, FL_ENOCONV, "tridiagonalisation: a cooperative wait was abandoned");
        }
    }
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_STEDC));
    int rc = fl_stedc_device(ctx, n, w, e, Z, ldz, leaf);
    if (rc) {
        if (info) info->index = FL_STAGE_STEDC;
        return rc;
    }
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_Q2));
    FL_HIP(ctx, bT2.alloc(sizeof(double) * fl_q2_t_elems(n, b, maxt)));
    FL_HIP(ctx, fl_q2_apply(s, n, b, bV2.as<double>(), btau2.as<double>(), maxt, bT2.as<double>(), Z, ldz, n));
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_Q1));
    FL_HIP(ctx, fl_q1_apply(s, n, b, bV1.as<double>(), n, bT1.as<double>(), Z, ldz, n, bwork.as<double>()));
    if (tm) FL_HIP(ctx, tm->mark(-1));
    FL_HIP(ctx, hipStreamSynchronize(s));
    return FL_OK;
}

// Mixed precision: both back-transforms (and, with fp32_band, the band
// reduction) on the FP32 matrix cores; the bulge chasing and the divide and
// conquer in FP64.  C is destroyed.
int fl_syevd_mixed_device(fl_ctx* ctx, int64_t n, double* C, int64_t ldc, int band, int fp32_band, double* w,
                          double* Z, int64_t ldz, fl_eig_info* info, int leaf, StageTimer* tm) {
    hipStream_t s = ctx->stream;
    const int b = clamp_band(n, band);
    const int64_t ldab = 2 * b + 1;
    const int64_t np = std::max<int64_t>(1, fl_sy2sb_panels(n, b));
    const int64_t maxt = fl_sb2st_maxt(n, b);
    const int64_t nsw = std::max<int64_t>(1, n - 2);
    DevBuf bA, bAB, bV1, bT1, btau1, bwork, bpart, bcnt, bV2, btau2, bprog, bT2, be;
    FL_HIP(ctx, bA.alloc(sizeof(float) * (size_t)n * n));
    double* ABp = band_buffer(ctx, sizeof(double) * ldab * n);
    if (!ABp) {
        FL_HIP(ctx, bAB.alloc(sizeof(double) * ldab * n));
        ABp = bAB.as<double>();
    }
    FL_HIP(ctx, bV1.alloc(sizeof(float) * (size_t)n * n));
    FL_HIP(ctx, hipMemsetAsync(bV1.p, 0, sizeof(float) * (size_t)n * n, s));  // Q1 reads above each panel
    FL_HIP(ctx, bT1.alloc(sizeof(float) * np * b * b));
    FL_HIP(ctx, btau1.alloc(sizeof(float) * (n + b)));
    FL_HIP(ctx, bwork.alloc(sizeof(float) * std::max<int64_t>(fl_sy2sb_work_elems(n, b), fl_q1_work_elems(n, b, n))));
    FL_HIP(ctx, bpart.alloc(sizeof(float) * fl_sy2sb_part_elems(n)));
    FL_HIP(ctx, bcnt.alloc(sizeof(unsigned) * np));
    FL_HIP(ctx, bV2.alloc(sizeof(double) * nsw * maxt * b));
    FL_HIP(ctx, btau2.alloc(sizeof(double) * nsw * maxt));
    FL_HIP(ctx, bprog.alloc(sizeof(int) * (2 * n + 2)));
    FL_HIP(ctx, be.alloc(sizeof(double) * (n + 1)));
    double* e = be.as<double>();
    float* A = bA.as<float>();
    int* abort_flag = bprog.as<int>() + 2 * n + 1;
    FL_HIP(ctx, hipMemsetAsync(abort_flag, 0, sizeof(int), s));

    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_SY2SB));
    if (fp32_band) {
        FL_HIP(ctx, fl_d2s(s, n, n, C, ldc, A, n));
        FL_HIP(ctx, fl_ssy2sb(s, n, b, A, n, bV1.as<float>(), n, bT1.as<float>(), btau1.as<float>(),
                              bwork.as<float>(), bpart.as<float>(), bcnt.as<unsigned>(), abort_flag));
        FL_HIP(ctx, fl_extract_band_f(s, n, b, A, n, ABp, ldab));
    } else {
        // FP64 band reduction; its block reflectors are rounded to FP32 for Q1
        DevBuf bV1d, bT1d, btau1d, bworkd, bpartd;
        FL_HIP(ctx, bV1d.alloc(sizeof(double) * (size_t)n * n));
        FL_HIP(ctx, hipMemsetAsync(bV1d.p, 0, sizeof(double) * (size_t)n * n, s));
        FL_HIP(ctx, bT1d.alloc(sizeof(double) * np * b * b));
        FL_HIP(ctx, btau1d.alloc(sizeof(double) * (n + b)));
        FL_HIP(ctx, bworkd.alloc(sizeof(double) * fl_sy2sb_work_elems(n, b)));
        FL_HIP(ctx, bpartd.alloc(sizeof(double) * fl_sy2sb_part_elems(n)));
        FL_HIP(ctx, fl_sy2sb(s, n, b, C, ldc, bV1d.as<double>(), n, bT1d.as<double>(), btau1d.as<double>(),
                             bworkd.as<double>(), bpartd.as<double>(), bcnt.as<unsigned>(), abort_flag));
        FL_HIP(ctx, fl_extract_band(s, n, b, C, ldc, ABp, ldab));
        FL_HIP(ctx, fl_d2s(s, n, n, bV1d.as<double>(), n, bV1.as<float>(), n));
        FL_HIP(ctx, fl_d2s(s, np * b, b, bT1d.as<double>(), np * b, bT1.as<float>(), np * b));
        FL_HIP(ctx, hipStreamSynchronize(s));  // the FP64 buffers are released at scope exit
    }
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_SB2ST));
    FL_HIP(ctx, fl_sb2st(s, n, b, ABp, ldab, w, e, bV2.as<double>(), btau2.as<double>(), bprog.as<int>(),
                         grid_for_sb2st(n, b), abort_flag));
    {
        int ab = 0;
        FL_HIP(ctx, hipMemcpyAsync(&ab, abort_flag, sizeof(int), hipMemcpyDeviceToHost, s));
        FL_HIP(ctx, hipStreamSynchronize(s));
        if (ab) {
            if (info) info->index = FL_STAGE_SB2ST;
            return fl_fail(ctx, FL_ENOCONV, "tridiagonalisation: a cooperative wait was abandoned");
        }
    }
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_STEDC));
    int rc = fl_stedc_device(ctx, n, w, e, Z, ldz, leaf);
    if (rc) {
        if (info) info->index = FL_STAGE_STEDC;
        return rc;
    }
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_Q2));
    float* Zf = A;  // the reduced matrix is no longer needed
    FL_HIP(ctx, fl_d2s(s, n, n, Z, ldz, Zf, n));
    FL_HIP(ctx, bT2.alloc(sizeof(float) * fl_q2_t_elems(n, b, maxt)));
    FL_HIP(ctx, fl_q2_apply_f(s, n, b, bV2.as<double>(), btau2.as<double>(), maxt, bT2.as<float>(), Zf, n, n));
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_Q1));
    FL_HIP(ctx, fl_q1_apply_f(s, n, b, bV1.as<float>(), n, bT1.as<float>(), Zf, n, n, bwork.as<float>()));
    FL_HIP(ctx, fl_s2d(s, n, n, Zf, n, Z, ldz));
    if (tm) FL_HIP(ctx, tm->mark(-1));
    FL_HIP(ctx, hipStreamSynchronize(s));
    return FL_OK;
}

extern "C" {

int fl_eigensolve(fl_op* op, int precision, const fl_eig_opts* opts, fl_eig_info* info) {
    if (!op) return FL_EINVAL;
    fl_ctx* ctx = op->ctx;
    if (precision != FL_FP64 && precision != FL_MIXED) return fl_fail(ctx, FL_EINVAL, "fl_eigensolve: bad precision");
    fl_eig_info local_info{};
    if (!info) info = &local_info;  // the refinement statistics are kept with the operator
    *info = fl_eig_info{};
    FL_HIP(ctx, hipSetDevice(ctx->device));
    const int64_t n = op->n, ld = op->ld;
    const int band = opts ? opts->band : 0;
    const int leaf = opts ? opts->leaf : 0;
    hipStream_t s = ctx->stream;
    DevBuf bL, bC, blinv, bwork, binfo;
    FL_HIP(ctx, bL.alloc(sizeof(double) * ld * n));
    FL_HIP(ctx, bC.alloc(sizeof(double) * ld * n));
    FL_HIP(ctx, blinv.alloc(sizeof(double) * fl_potrf_linv_elems(n)));
    FL_HIP(ctx, bwork.alloc(sizeof(double) * fl_trsm_work_elems(n, n)));
    FL_HIP(ctx, binfo.alloc(sizeof(int64_t)));
    if (!op->theta || !op->V || !op->logtheta) {
        if (!op->theta) FL_HIP(ctx, hipMalloc(&op->theta, sizeof(double) * n));
        if (!op->logtheta) FL_HIP(ctx, hipMalloc(&op->logtheta, sizeof(double) * n));
        if (!op->V) FL_HIP(ctx, hipMalloc(&op->V, sizeof(double) * ld * n));
    }
    op->has_eig = 0;
    double* L = bL.as<double>();
    double* C = bC.as<double>();
    StageTimer tm(s);
    FL_HIP(ctx, tm.mark(FL_STAGE_POTRF));
    FL_HIP(ctx, hipMemcpyAsync(L, op->M, sizeof(double) * ld * n, hipMemcpyDeviceToDevice, s));
    FL_HIP(ctx, hipMemsetAsync(binfo.p, 0, sizeof(int64_t), s));
    FL_HIP(ctx, fl_potrf(s, n, L, ld, blinv.as<double>(), binfo.as<int64_t>(), bwork.as<double>()));
    int64_t piv = 0;
    FL_HIP(ctx, hipMemcpyAsync(&piv, binfo.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FL_HIP(ctx, hipStreamSynchronize(s));
    if (piv) {
        if (info) {
            info->status = FL_ENOTSPD;
            info->index = piv;
        }
        return fl_fail(ctx, FL_ENOTSPD, "fl_eigensolve: M is not positive definite at pivot " + std::to_string(piv));
    }
    FL_HIP(ctx, tm.mark(FL_STAGE_SYGST));
    // With a sparse K: X = L^-1 explicitly (in place of L), Y = K X^T as a
    // sparse product, and only the lower triangle of C = X Y, skipping X's
    // zero tiles (about half the work of two dense triangular solves);
    // V = X^T Z at the end is one GEMM.  Dense K: two triangular solves.
    const bool sparse = op->rowptr && op->kval && op->nnz <= (n * n) / 64;
    DevBuf bXt, bY;
    int rc = FL_OK;
    if (sparse) {
        FL_HIP(ctx, bXt.alloc(sizeof(double) * (size_t)n * n));
        FL_HIP(ctx, bY.alloc(sizeof(double) * (size_t)n * n));
        double* Xt = bXt.as<double>();
        double* Y = bY.as<double>();
        FL_HIP(ctx, fl_trtri_inplace(s, n, L, ld, blinv.as<double>(), Y));
        FL_HIP(ctx, fl_transpose(s, n, n, L, ld, Xt, n));
        FL_HIP(ctx, fl_spmm_csr(s, n, op->rowptr, op->colidx, op->kval, n, Xt, n, Y, n));
        FL_HIP(ctx, fl_dgemm_tri(s, 0, 0, n, n, n, 1.0, L, ld, Y, n, 0.0, C, ld, 1, FL_KT_A_LOWER));
        FL_HIP(ctx, fl_mirror_lower(s, n, C, ld));
    } else {
        FL_HIP(ctx, hipMemcpyAsync(C, op->K, sizeof(double) * ld * n, hipMemcpyDeviceToDevice, s));
        rc = fl_sygst_device(ctx, n, L, ld, blinv.as<double>(), C, ld, bwork.as<double>());
        if (rc) return rc;
    }
    if (precision == FL_MIXED)
        rc = fl_syevd_mixed_device(ctx, n, C, ld, band, opts ? (opts->mixed_flags & FL_MIXED_FP32_BAND) : 0,
                                   op->theta, op->V, ld, info, leaf, &tm);
    else
        rc = fl_syevd_device(ctx, n, C, ld, band, op->theta, op->V, ld, info, leaf, &tm);
    if (rc) {
        if (info) info->status = rc;
        return rc;
    }
    FL_HIP(ctx, tm.mark(FL_STAGE_TRSM));
    if (sparse) {
        // V = X^T Z (X^T upper triangular)
        double* Y = bY.as<double>();
        FL_HIP(ctx, fl_dgemm_tri(s, 1, 0, n, n, n, 1.0, L, ld, op->V, ld, 0.0, Y, n, 0, FL_KT_A_UPPER));
        FL_HIP(ctx, fl_copy_matrix(s, n, n, Y, n, op->V, ld));
    } else {
        FL_HIP(ctx, fl_trsm_llt(s, n, n, L, ld, blinv.as<double>(), op->V, ld, bwork.as<double>()));
    }
    // refinement: by default two steps after FP32 back-transforms (the first
    // meets the eigenvalue and orthonormality targets; the second removes the
    // second-order error between close low modes, which dominates the
    // fractional solutions), three after an FP32 band reduction (early exit
    // at tol), none in FP64 mode
    const bool fp32_band = opts && (opts->mixed_flags & FL_MIXED_FP32_BAND);
    int iters = (opts && opts->refine_max_iters >= 0) ? opts->refine_max_iters
                                                      : (precision == FL_MIXED ? (fp32_band ? 3 : 2) : 0);
    double tol = (opts && opts->refine_tol > 0.0) ? opts->refine_tol : 1e-13;
    if (iters > 0) {
        FL_HIP(ctx, hipStreamSynchronize(s));  // the TRSM above still reads L
        bL.release();  // L and C are not needed any more: room for the refinement buffers
        bC.release();
        FL_HIP(ctx, tm.mark(FL_STAGE_REFINE));
        rc = fl_refine_device(ctx, op, op->theta, op->V, ld, iters, tol, info, 0);
        if (rc) {
            if (info) {
                info->status = rc;
                info->index = FL_STAGE_REFINE;
            }
            return rc;
        }
    }
    if (iters == 0 && op->rowptr && op->kval) {
        // no refinement: the eigenvalues become the Rayleigh quotients of the
        // computed vectors with the original pencil (the solver's normwise
        // error, about eps ||C||, is large relative to the smallest
        // eigenvalues; the quotients are accurate to second order)
        FL_HIP(ctx, hipStreamSynchronize(s));
        bL.release();
        bC.release();
        FL_HIP(ctx, tm.mark(FL_STAGE_REFINE));
        rc = fl_rayleigh_device(ctx, op, op->theta, op->V, ld);
        if (rc) {
            if (info) {
                info->status = rc;
                info->index = FL_STAGE_REFINE;
            }
            return rc;
        }
    }
    FL_HIP(ctx, fl_log_kernel(s, n, op->theta, op->logtheta));
    FL_HIP(ctx, tm.mark(-1));
    FL_HIP(ctx, hipStreamSynchronize(s));
    if (info) {
        tm.collect(info);
        info->flops_nominal = 9.0 * (double)n * (double)n * (double)n;
    }
    double th0 = 0.0;
    FL_HIP(ctx, hipMemcpy(&th0, op->theta, sizeof(double), hipMemcpyDeviceToHost));
    if (!(th0 > 0.0)) {
        if (info) info->status = FL_EINVAL;
        return fl_fail(ctx, FL_EINVAL, "fl_eigensolve: smallest eigenvalue is not positive");
    }
    op->has_eig = 1;
    op->eig_precision = precision;
    op->refine_iters = info->refine_iters;
    op->refine_resid = info->refine_resid;
    return FL_OK;
}

int fl_dstedc(fl_ctx* ctx, int64_t n, double* d, double* e, double* Z, int64_t ldz) {
    if (!ctx) return FL_EINVAL;
    if (n <= 0 || !d || !Z || ldz < n || (n > 1 && !e)) return fl_fail(ctx, FL_EINVAL, "fl_dstedc: bad arguments");
    FL_HIP(ctx, hipSetDevice(ctx->device));
    DevBuf be;
    FL_HIP(ctx, be.alloc(sizeof(double) * (n + 1)));
    FL_HIP(ctx, hipMemsetAsync(be.p, 0, sizeof(double) * (n + 1), ctx->stream));
    if (n > 1)
        FL_HIP(ctx, hipMemcpyAsync(be.p, e, sizeof(double) * (n - 1), hipMemcpyDeviceToDevice, ctx->stream));
    return fl_stedc_device(ctx, n, d, be.as<double>(), Z, ldz, 0);
}

int fl_dsyevd(fl_ctx* ctx, int64_t n, double* A, int64_t lda, int band, double* w, double* Z, int64_t ldz) {
    if (!ctx) return FL_EINVAL;
    if (n <= 0 || !A || !w || !Z || lda < n || ldz < n) return fl_fail(ctx, FL_EINVAL, "fl_dsyevd: bad arguments");
    FL_HIP(ctx, hipSetDevice(ctx->device));
    return fl_syevd_device(ctx, n, A, lda, band, w, Z, ldz, nullptr, 0, nullptr);
}

int fl_dsytrd_2stage(fl_ctx* ctx, int64_t n, double* A, int64_t lda, int band, double* d, double* e, double* Q,
                     int64_t ldq) {
    if (!ctx) return FL_EINVAL;
    if (n <= 0 || !A || !d || !e || lda < n || (Q && ldq < n)) return fl_fail(ctx, FL_EINVAL, "fl_dsytrd_2stage: bad arguments");
    FL_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int b = clamp_band(n, band);
    const int64_t ldab = 2 * b + 1;
    const int64_t np = std::max<int64_t>(1, fl_sy2sb_panels(n, b));
    const int64_t maxt = fl_sb2st_maxt(n, b);
    const int64_t nsw = std::max<int64_t>(1, n - 2);
    DevBuf bAB, bV1, bT1, btau1, bwork, bpart, bcnt, bV2, btau2, bprog, bT2, be;
    double* ABp = band_buffer(ctx, sizeof(double) * ldab * n);
    if (!ABp) {
        FL_HIP(ctx, bAB.alloc(sizeof(double) * ldab * n));
        ABp = bAB.as<double>();
    }
    FL_HIP(ctx, bV1.alloc(sizeof(double) * (size_t)n * n));
    FL_HIP(ctx, hipMemsetAsync(bV1.p, 0, sizeof(double) * (size_t)n * n, s));  // Q1 reads above each panel
    FL_HIP(ctx, bT1.alloc(sizeof(double) * np * b * b));
    FL_HIP(ctx, btau1.alloc(sizeof(double) * (n + b)));
    FL_HIP(ctx, bwork.alloc(sizeof(double) * std::max<int64_t>(fl_sy2sb_work_elems(n, b), fl_q1_work_elems(n, b, n))));
    FL_HIP(ctx, bpart.alloc(sizeof(double) * fl_sy2sb_part_elems(n)));
    FL_HIP(ctx, bcnt.alloc(sizeof(unsigned) * np));
    FL_HIP(ctx, bV2.alloc(sizeof(double) * nsw * maxt * b));
    FL_HIP(ctx, btau2.alloc(sizeof(double) * nsw * maxt));
    FL_HIP(ctx, bprog.alloc(sizeof(int) * (2 * n + 2)));
    FL_HIP(ctx, be.alloc(sizeof(double) * (n + 1)));
    int* abort_flag = bprog.as<int>() + 2 * n + 1;
    FL_HIP(ctx, hipMemsetAsync(abort_flag, 0, sizeof(int), s));
    FL_HIP(ctx, fl_sy2sb(s, n, b, A, lda, bV1.as<double>(), n, bT1.as<double>(), btau1.as<double>(), bwork.as<double>(),
                         bpart.as<double>(), bcnt.as<unsigned>(), abort_flag));
    FL_HIP(ctx, fl_extract_band(s, n, b, A, lda, ABp, ldab));
    FL_HIP(ctx, fl_sb2st(s, n, b, ABp, ldab, d, be.as<double>(), bV2.as<double>(), btau2.as<double>(),
                         bprog.as<int>(), grid_for_sb2st(n, b), abort_flag));
    {
        int ab = 0;
        FL_HIP(ctx, hipMemcpyAsync(&ab, abort_flag, sizeof(int), hipMemcpyDeviceToHost, s));
        FL_HIP(ctx, hipStreamSynchronize(s));
        if (ab) return fl_fail(ctx, FL_ENOCONV, "tridiagonalisation: a cooperative wait was abandoned");
    }
    if (n > 1) FL_HIP(ctx, hipMemcpyAsync(e, be.p, sizeof(double) * (n - 1), hipMemcpyDeviceToDevice, s));
    if (Q) {
        FL_HIP(ctx, fl_set_identity(s, n, Q, ldq));
        FL_HIP(ctx, bT2.alloc(sizeof(double) * fl_q2_t_elems(n, b, maxt)));
        FL_HIP(ctx, fl_q2_apply(s, n, b, bV2.as<double>(), btau2.as<double>(), maxt, bT2.as<double>(), Q, ldq, n));
        FL_HIP(ctx, fl_q1_apply(s, n, b, bV1.as<double>(), n, bT1.as<double>(), Q, ldq, n, bwork.as<double>()));
    }
    FL_HIP(ctx, hipStreamSynchronize(s));
    return FL_OK;
}

}  // extern "C"
