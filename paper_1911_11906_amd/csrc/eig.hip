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
                    double* tau1, double* work, double* part, int* abort);
int64_t fl_sy2sb_work_elems(int64_t n, int b);
int64_t fl_sy2sb_part_elems(int64_t n);
hipError_t fl_extract_band(hipStream_t s, int64_t n, int b, const double* A, int64_t lda, double* AB, int64_t ldab);
// sb2st.hip
int64_t fl_sb2st_maxt(int64_t n, int b);
bool fl_sb2st_ring_fits(int64_t n, int b);
int64_t fl_sb2st_ring_msg_elems(int64_t n);
hipError_t fl_sb2st_ring(hipStream_t s, int64_t n, const double* AB, int64_t ldab, double* d, double* e, double* V2,
                         double* tau2, double* RM, int* abort);
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
                     float* tau1, float* work, float* part, int* abort);
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

// The two-stage tridiagonalisation shared by every eigensolve entry point:
// band reduction (FP64 or FP32) -> band (FP64) -> bulge chase (FP64), and the
// two back-transforms Z := Q1 Q2 Z in the precision of Z.  Owns every buffer
// of the sequence; V1 (the band reduction's block reflectors) is kept in the
// precision of the back-transforms that will read it (FP64 reflectors are
// rounded to FP32 when the back-transforms run in FP32).
struct TwoStage {
    fl_ctx* ctx;
    hipStream_t s;
    int64_t n;
    int b;
    int64_t ldab, np, maxt, nsw;
    DevBuf bAB, bV2, btau2, bprog, be, bT2;
    DevBuf bV1, bT1;  // reflectors for the back-transforms (FP64 or FP32)
    bool q_fp32 = false;
    double* AB = nullptr;
    int* abort_flag = nullptr;

    TwoStage(fl_ctx* c, int64_t n_, int band) : ctx(c), s(c->stream), n(n_), b(clamp_band(n_, band)) {
        ldab = 2 * (int64_t)b + 1;
        np = std::max<int64_t>(1, fl_sy2sb_panels(n, b));
        maxt = fl_sb2st_maxt(n, b);
        nsw = std::max<int64_t>(1, n - 2);
    }
    double* e() const { return be.as<double>(); }

    // common buffers; q_in_fp32: the back-transforms will run in FP32
    int init(bool q_in_fp32) {
        q_fp32 = q_in_fp32;
        AB = band_buffer(ctx, sizeof(double) * ldab * n);
        if (!AB) {
            FL_HIP(ctx, bAB.alloc(sizeof(double) * ldab * n));
            AB = bAB.as<double>();
        }
        const size_t esz = q_fp32 ? sizeof(float) : sizeof(double);
        FL_HIP(ctx, bV1.alloc(esz * (size_t)n * n));
        FL_HIP(ctx, hipMemsetAsync(bV1.p, 0, esz * (size_t)n * n, s));  // Q1 reads above each panel
        FL_HIP(ctx, bT1.alloc(esz * np * b * b));
        FL_HIP(ctx, bV2.alloc(sizeof(double) * nsw * maxt * b));
        FL_HIP(ctx, btau2.alloc(sizeof(double) * nsw * maxt));
        FL_HIP(ctx, bprog.alloc(sizeof(int) * (2 * n + 2)));
        FL_HIP(ctx, be.alloc(sizeof(double) * (n + 1)));
        abort_flag = bprog.as<int>() + 2 * n + 1;
        FL_HIP(ctx, hipMemsetAsync(abort_flag, 0, sizeof(int), s));
        return FL_OK;
    }

    // A (full symmetric storage, FP64, destroyed) -> band; the reflectors are
    // kept for the back-transforms (rounded to FP32 if they run in FP32)
    int reduce(double* A, int64_t lda) {
        DevBuf tau, work, part, V1d, T1d;
        FL_HIP(ctx, tau.alloc(sizeof(double) * (n + b)));
        FL_HIP(ctx, work.alloc(sizeof(double) * fl_sy2sb_work_elems(n, b)));
        FL_HIP(ctx, part.alloc(sizeof(double) * fl_sy2sb_part_elems(n)));
        double* V1 = bV1.as<double>();
        double* T1 = bT1.as<double>();
        if (q_fp32) {
            FL_HIP(ctx, V1d.alloc(sizeof(double) * (size_t)n * n));
            FL_HIP(ctx, hipMemsetAsync(V1d.p, 0, sizeof(double) * (size_t)n * n, s));
            FL_HIP(ctx, T1d.alloc(sizeof(double) * np * b * b));
            V1 = V1d.as<double>();
            T1 = T1d.as<double>();
        }
        FL_HIP(ctx, fl_sy2sb(s, n, b, A, lda, V1, n, T1, tau.as<double>(), work.as<double>(), part.as<double>(),
                             abort_flag));
        FL_HIP(ctx, fl_extract_band(s, n, b, A, lda, AB, ldab));
        if (q_fp32) {
            FL_HIP(ctx, fl_d2s(s, n, n, V1, n, bV1.as<float>(), n));
            FL_HIP(ctx, fl_d2s(s, np * b, b, T1, np * b, bT1.as<float>(), np * b));
        }
        FL_HIP(ctx, hipStreamSynchronize(s));  // the scoped buffers are released at return
        return check_abort("band reduction");
    }

    // FL_ENOCONV if a cooperative wait of the last stage was abandoned (the
    // flag is cleared for the next stage)
    int check_abort(const char* stage) {
        int ab = 0;
        FL_HIP(ctx, hipMemcpyAsync(&ab, abort_flag, sizeof(int), hipMemcpyDeviceToHost, s));
        FL_HIP(ctx, hipStreamSynchronize(s));
        if (!ab) return FL_OK;
        FL_HIP(ctx, hipMemsetAsync(abort_flag, 0, sizeof(int), s));
        return fl_fail(ctx, FL_ENOCONV, std::string(stage) + ": a cooperative wait was abandoned");
    }

    // A (full symmetric storage, FP32, destroyed) -> band; FP32 reflectors
    int reduce(float* A, int64_t lda) {
        if (!q_fp32) return fl_fail(ctx, FL_EINVAL, "two-stage: an FP32 band reduction needs FP32 back-transforms");
        DevBuf tau, work, part;
        FL_HIP(ctx, tau.alloc(sizeof(float) * (n + b)));
        FL_HIP(ctx, work.alloc(sizeof(float) * fl_sy2sb_work_elems(n, b)));
        FL_HIP(ctx, part.alloc(sizeof(float) * fl_sy2sb_part_elems(n)));
        FL_HIP(ctx, fl_ssy2sb(s, n, b, A, lda, bV1.as<float>(), n, bT1.as<float>(), tau.as<float>(),
                              work.as<float>(), part.as<float>(), abort_flag));
        FL_HIP(ctx, fl_extract_band_f(s, n, b, A, lda, AB, ldab));
        FL_HIP(ctx, hipStreamSynchronize(s));
        return check_abort("band reduction");
    }

    // band -> d (n), e() (n - 1), reflectors V2; FL_ENOCONV if a cooperative
    // wait of the band reduction or of the bulge chase was abandoned
    // (the stationary chase when b = 64 and every block column fits on the
    // device at once, else the sweep-per-workgroup chase)
    int chase(double* d, fl_eig_info* info) {
        if (fl_sb2st_ring_fits(n, b)) {
            DevBuf rm;
            FL_HIP(ctx, rm.alloc(sizeof(double) * fl_sb2st_ring_msg_elems(n)));
            FL_HIP(ctx, fl_sb2st_ring(s, n, AB, ldab, d, e(), bV2.as<double>(), btau2.as<double>(), rm.as<double>(),
                                      abort_flag));
            FL_HIP(ctx, hipStreamSynchronize(s));  // rm is released at return
        } else {
            FL_HIP(ctx, fl_sb2st(s, n, b, AB, ldab, d, e(), bV2.as<double>(), btau2.as<double>(), bprog.as<int>(),
                                 grid_for_sb2st(n, b), abort_flag));
        }
        int ab = 0;
        FL_HIP(ctx, hipMemcpyAsync(&ab, abort_flag, sizeof(int), hipMemcpyDeviceToHost, s));
        FL_HIP(ctx, hipStreamSynchronize(s));
        if (ab) {
            if (info) info->index = FL_STAGE_SB2ST;
            return fl_fail(ctx, FL_ENOCONV, "tridiagonalisation: a cooperative wait was abandoned");
        }
        return FL_OK;
    }

    int apply_q2(double* Z, int64_t ldz, int64_t ncols) {
        FL_HIP(ctx, bT2.alloc(sizeof(double) * fl_q2_t_elems(n, b, maxt)));
        FL_HIP(ctx, fl_q2_apply(s, n, b, bV2.as<double>(), btau2.as<double>(), maxt, bT2.as<double>(), Z, ldz, ncols));
        return FL_OK;
    }
    int apply_q2(float* Z, int64_t ldz, int64_t ncols) {
        FL_HIP(ctx, bT2.alloc(sizeof(float) * fl_q2_t_elems(n, b, maxt)));
        FL_HIP(ctx, fl_q2_apply_f(s, n, b, bV2.as<double>(), btau2.as<double>(), maxt, bT2.as<float>(), Z, ldz, ncols));
        return FL_OK;
    }
    int apply_q1(double* Z, int64_t ldz, int64_t ncols) {
        if (q_fp32) return fl_fail(ctx, FL_EINVAL, "two-stage: FP32 reflectors applied to FP64 vectors");
        DevBuf work;
        FL_HIP(ctx, work.alloc(sizeof(double) * fl_q1_work_elems(n, b, ncols)));
        FL_HIP(ctx, fl_q1_apply(s, n, b, bV1.as<double>(), n, bT1.as<double>(), Z, ldz, ncols, work.as<double>()));
        FL_HIP(ctx, hipStreamSynchronize(s));
        return FL_OK;
    }
    int apply_q1(float* Z, int64_t ldz, int64_t ncols) {
        if (!q_fp32) return fl_fail(ctx, FL_EINVAL, "two-stage: FP64 reflectors applied to FP32 vectors");
        DevBuf work;
        FL_HIP(ctx, work.alloc(sizeof(float) * fl_q1_work_elems(n, b, ncols)));
        FL_HIP(ctx, fl_q1_apply_f(s, n, b, bV1.as<float>(), n, bT1.as<float>(), Z, ldz, ncols, work.as<float>()));
        FL_HIP(ctx, hipStreamSynchronize(s));
        return FL_OK;
    }
};

}  // namespace

// Two-stage tridiagonalisation + D&C + back-transforms of the symmetric A
// (full storage, destroyed).  w (n) ascending, Z (n x n, ld ldz).
int fl_syevd_device(fl_ctx* ctx, int64_t n, double* A, int64_t lda, int band, double* w, double* Z, int64_t ldz,
                    fl_eig_info* info, int leaf, StageTimer* tm) {
    TwoStage ts(ctx, n, band);
    int rc;
    if ((rc = ts.init(false))) return rc;
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_SY2SB));
    if ((rc = ts.reduce(A, lda))) {
        if (info) info->index = FL_STAGE_SY2SB;
        return rc;
    }
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_SB2ST));
    if ((rc = ts.chase(w, info))) return rc;
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_STEDC));
    if ((rc = fl_stedc_device(ctx, n, w, ts.e(), Z, ldz, leaf))) {
        if (info) info->index = FL_STAGE_STEDC;
        return rc;
    }
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_Q2));
    if ((rc = ts.apply_q2(Z, ldz, n))) return rc;
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_Q1));
    if ((rc = ts.apply_q1(Z, ldz, n))) return rc;
    if (tm) FL_HIP(ctx, tm->mark(-1));
    FL_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return FL_OK;
}

// Mixed precision: both back-transforms (and, with fp32_band, the band
// reduction) on the FP32 matrix cores; the bulge chasing and the divide and
// conquer in FP64.  C is destroyed.
int fl_syevd_mixed_device(fl_ctx* ctx, int64_t n, double* C, int64_t ldc, int band, int fp32_band, double* w,
                          double* Z, int64_t ldz, fl_eig_info* info, int leaf, StageTimer* tm) {
    hipStream_t s = ctx->stream;
    TwoStage ts(ctx, n, band);
    DevBuf bA;  // FP32 copy of C for an FP32 band reduction, then the FP32 vectors
    FL_HIP(ctx, bA.alloc(sizeof(float) * (size_t)n * n));
    float* Af = bA.as<float>();
    int rc;
    if ((rc = ts.init(true))) return rc;
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_SY2SB));
    if (fp32_band) {
        FL_HIP(ctx, fl_d2s(s, n, n, C, ldc, Af, n));
        rc = ts.reduce(Af, n);
    } else {
        rc = ts.reduce(C, ldc);
    }
    if (rc) {
        if (info) info->index = FL_STAGE_SY2SB;
        return rc;
    }
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_SB2ST));
    if ((rc = ts.chase(w, info))) return rc;
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_STEDC));
    if ((rc = fl_stedc_device(ctx, n, w, ts.e(), Z, ldz, leaf))) {
        if (info) info->index = FL_STAGE_STEDC;
        return rc;
    }
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_Q2));
    FL_HIP(ctx, fl_d2s(s, n, n, Z, ldz, Af, n));  // the reduced matrix is no longer needed
    if ((rc = ts.apply_q2(Af, n, n))) return rc;
    if (tm) FL_HIP(ctx, tm->mark(FL_STAGE_Q1));
    if ((rc = ts.apply_q1(Af, n, n))) return rc;
    FL_HIP(ctx, fl_s2d(s, n, n, Af, n, Z, ldz));
    if (tm) FL_HIP(ctx, tm->mark(-1));
    FL_HIP(ctx, hipStreamSynchronize(s));
    return FL_OK;
}

extern "C" {

int fl_eigensolve(fl_op* op, int precision, const fl_eig_opts* opts, fl_eig_info* info) {
    if (!op) return FL_EINVAL;
    fl_ctx* ctx = op->ctx;
    if (precision != FL_FP64 && precision != FL_MIXED) return fl_fail(ctx, FL_EINVAL, "fl_eigensolve: bad precision");
    if (!op->K || !op->M)
        return fl_fail(ctx, FL_ESTATE, "fl_eigensolve: the operator holds no dense pencil (assembled sparse)");
    fl_eig_info local_info{};
    if (!info) info = &local_info;  // the refinement statistics are kept with the operator
    *info = fl_eig_info{};
    FL_HIP(ctx, hipSetDevice(ctx->device));
    const int64_t n = op->n, ld = op->ld;
    const int band = opts ? opts->band : 0;
    const int leaf = opts ? opts->leaf : 0;
    hipStream_t s = ctx->stream;
    DevBuf bL, bC, blinv, bwork, binfo, bpan, bprob;
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
    // A mass matrix whose pattern is banded (FEM: half-bandwidth ~ the
    // number of nodes across the mesh in its own numbering) keeps its band in
    // the factor: factor and triangular solves then run on the q block rows
    // below each 128 x 128 diagonal block only.
    int64_t mbw = -1;
    {
        int rcb = fl_pattern_bandwidth(op, &mbw);
        if (rcb) return rcb;
    }
    const int64_t qband = mbw >= 0 ? FL_DIV_UP(std::max<int64_t>(mbw, 1), 128) : -1;
    const bool banded = qband > 0 && (qband + 1) * 128 <= n / 4;
    StageTimer tm(s);
    FL_HIP(ctx, tm.mark(FL_STAGE_POTRF));
    FL_HIP(ctx, hipMemcpyAsync(L, op->M, sizeof(double) * ld * n, hipMemcpyDeviceToDevice, s));
    FL_HIP(ctx, hipMemsetAsync(binfo.p, 0, sizeof(int64_t), s));
    if (banded)
        FL_HIP(ctx, fl_potrf_band(s, n, qband, L, ld, blinv.as<double>(), binfo.as<int64_t>(), bwork.as<double>()));
    else
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
    const bool sparse = !banded && op->rowptr && op->kval && op->nnz <= (n * n) / 64;
    DevBuf bXt, bY;
    int rc = FL_OK;
    if (banded) {
        // W = L^-1 K, then C = L^-1 W^T (= L^-1 K L^-T, symmetric): two
        // banded substitutions, strip-parallel (the first skips the blocks
        // where W is zero: K shares M's pattern, so row r of W ends at
        // column r + bw); the lower triangle is mirrored so that C is
        // exactly symmetric
        FL_HIP(ctx, bY.alloc(sizeof(double) * (size_t)n * n));
        double* Y = bY.as<double>();
        FL_HIP(ctx, bpan.alloc(sizeof(double) * (size_t)fl_band_panel_elems(n, qband)));
        FL_HIP(ctx, bprob.alloc(sizeof(GemmProblem) * (size_t)FL_DIV_UP(n, 128)));
        FL_HIP(ctx, fl_band_panels(s, n, qband, L, ld, blinv.as<double>(), bpan.as<double>(), 0,
                                   bprob.as<GemmProblem>()));
        FL_HIP(ctx, hipMemcpyAsync(C, op->K, sizeof(double) * ld * n, hipMemcpyDeviceToDevice, s));
        FL_HIP(ctx, fl_band_solve(s, n, qband, bpan.as<double>(), C, ld, n, 0, mbw));
        FL_HIP(ctx, fl_transpose(s, n, n, C, ld, Y, n));
        FL_HIP(ctx, fl_band_solve(s, n, qband, bpan.as<double>(), Y, n, n, 0, -1));
        FL_HIP(ctx, fl_copy_matrix(s, n, n, Y, n, C, ld));
        FL_HIP(ctx, fl_mirror_lower(s, n, C, ld));
        FL_HIP(ctx, hipStreamSynchronize(s));
        bY.release();
    } else if (sparse) {
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
    if (banded) {
        FL_HIP(ctx, fl_band_panels(s, n, qband, L, ld, blinv.as<double>(), bpan.as<double>(), 1,
                                   bprob.as<GemmProblem>()));
        FL_HIP(ctx, fl_band_solve(s, n, qband, bpan.as<double>(), op->V, ld, n, 1, -1));
    } else if (sparse) {
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
    TwoStage ts(ctx, n, band);
    int rc;
    if ((rc = ts.init(false)) || (rc = ts.reduce(A, lda)) || (rc = ts.chase(d, nullptr))) return rc;
    if (n > 1) FL_HIP(ctx, hipMemcpyAsync(e, ts.e(), sizeof(double) * (n - 1), hipMemcpyDeviceToDevice, s));
    if (Q) {
        FL_HIP(ctx, fl_set_identity(s, n, Q, ldq));
        if ((rc = ts.apply_q2(Q, ldq, n)) || (rc = ts.apply_q1(Q, ldq, n))) return rc;
    }
    FL_HIP(ctx, hipStreamSynchronize(s));
    return FL_OK;
}

}  // extern "C"
