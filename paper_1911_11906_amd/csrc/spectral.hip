// Entry points of the spectral application (Section "Method": the equation
// for v of the fractional Poisson problem, and the solution of the diffusion
// equation, equation diffusion_solution), their adjoints, and the replay of a
// captured application graph.
//
//   G = M F (CSR SpMM),  C = V^T G (MFMA GEMM),  W = spectral weights,
//   U[:, j + i nf] = V (W[:, i] o C[:, j])  (one fused scaled GEMM).
//
// Each operator keeps one workspace per stream, so calls queued on different
// streams never share intermediate buffers (products that split along k use
// a buffer owned by their stream as well).
#include <cmath>
#include <cstring>
#include <string>
#include <vector>
#include "internal.h"

struct ApplyGraph {
    // key: every argument of the call
    int kind = 0;
    int64_t nf = 0, ldf = 0, na = 0, ldu = 0;
    int paired = 0;
    const double* F = nullptr;
    double* U = nullptr;
    std::vector<double> alpha, sprm;
    // captured sequence and the workspace its kernels use
    hipGraphExec_t exec = nullptr;
    double* ws = nullptr;
    uint64_t last_use = 0;
};

namespace {

constexpr size_t MAX_GRAPHS_PER_OP = 8;

int set_device(fl_ctx* ctx) {
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fl_fail(ctx, FL_EHIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    return FL_OK;
}

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return s && hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// Workspace of at least `bytes` for stream s.  Growing it waits for the
// stream's queued work (which may still read the old buffer) first; inside a
// graph capture nothing may be allocated, so a missing or short workspace is
// an error there.
int op_ws(fl_op* op, hipStream_t s, size_t bytes, double** out) {
    fl_ctx* ctx = op->ctx;
    OpWs* w = nullptr;
    for (OpWs& x : op->ws)
        if (x.s == s) w = &x;
    if (w && w->bytes >= bytes) {
        *out = w->p;
        return FL_OK;
    }
    if (capturing(s))
        return fl_fail(ctx, FL_ESTATE, "spectral application: workspace must be reserved (one eager call on this "
                                       "stream) before graph capture");
    if (w) {
        FL_HIP(ctx, hipStreamSynchronize(s));
        (void)hipFree(w->p);
        w->p = nullptr;
        w->bytes = 0;
    } else {
        op->ws.push_back(OpWs{s, nullptr, 0});
        w = &op->ws.back();
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes > 0 ? bytes : 8) != hipSuccess) {
        (void)hipGetLastError();
        return fl_fail(ctx, FL_ENOMEM, "spectral application: workspace allocation of " + std::to_string(bytes) +
                                           " bytes failed");
    }
    w->p = static_cast<double*>(p);
    w->bytes = bytes;
    *out = w->p;
    return FL_OK;
}

int check_params(fl_ctx* ctx, const char* who, int64_t count, const double* alpha, const double* t,
                 const double* mu) {
    for (int64_t i = 0; i < count; ++i) {
        if (!std::isfinite(alpha[i]) || alpha[i] < 0.0 || alpha[i] > 2.0)
            return fl_fail(ctx, FL_EINVAL, std::string(who) + ": alpha must lie in [0, 2]");
        if (t && (!std::isfinite(t[i]) || t[i] < 0.0))
            return fl_fail(ctx, FL_EINVAL, std::string(who) + ": t must be finite and >= 0");
        if (mu && (!std::isfinite(mu[i]) || mu[i] < 0.0))
            return fl_fail(ctx, FL_EINVAL, std::string(who) + ": mu must be finite and >= 0");
    }
    return FL_OK;
}

WeightArgs chunk_args(int kind, const double* alpha, const double* sprm, int64_t i0, int64_t count) {
    WeightArgs a{};
    a.kind = kind;
    a.count = (int)std::min<int64_t>(FL_WCHUNK, count - i0);
    for (int i = 0; i < a.count; ++i) {
        a.alpha[i] = alpha[i0 + i];
        a.s[i] = sprm ? sprm[i0 + i] : 0.0;
    }
    return a;
}

hipError_t queue_weights(const fl_op* op, hipStream_t s, int kind, const double* alpha, const double* sprm,
                         int64_t count, double* W) {
    for (int64_t i0 = 0; i0 < count; i0 += FL_WCHUNK) {
        hipError_t e = fl_weights(s, op->n, op->logtheta, chunk_args(kind, alpha, sprm, i0, count), W + i0 * op->n,
                                  op->n);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Adjoint of the paired map, shared by both weight families.  GU = dL/dU
// (device n x nb); GF = M V (W o V^T GU); ga, gs: host, per-column
// derivatives with respect to alpha and to s = mu t (diffusion only).
int grad_spectral(fl_op* op, const char* who, int kind, int64_t nb, const double* F, int64_t ldf,
                  const double* alpha, const double* sprm, const double* GU, int64_t ldgu, double* GF,
                  int64_t ldgf, double* ga, double* gs) {
    fl_ctx* ctx = op->ctx;
    const int64_t n = op->n;
    const bool want_param = ga || gs;
    hipStream_t s = ctx->stream;
    // workspace: P | C | G | W | Y (n x nb each) | ga | gs (nb each)
    double* ws = nullptr;
    int rc = op_ws(op, s, ((size_t)5 * n * nb + 2 * nb) * 8, &ws);
    if (rc) return rc;
    double* P = ws;
    double* C = P + (size_t)n * nb;
    double* G = C + (size_t)n * nb;
    double* W = G + (size_t)n * nb;
    double* Y = W + (size_t)n * nb;
    double* dga = Y + (size_t)n * nb;
    double* dgs = dga + nb;
    FL_HIP(ctx, fl_dgemm(s, 1, 0, n, nb, n, 1.0, op->V, op->ld, GU, ldgu, 0.0, P, n));
    FL_HIP(ctx, queue_weights(op, s, kind, alpha, sprm, nb, W));
    if (want_param) {
        FL_HIP(ctx, fl_spmm_csr(s, n, op->rowptr, op->colidx, op->mval, nb, F, ldf, G, n));
        FL_HIP(ctx, fl_dgemm(s, 1, 0, n, nb, n, 1.0, op->V, op->ld, G, n, 0.0, C, n));
        for (int64_t i0 = 0; i0 < nb; i0 += FL_WCHUNK)
            FL_HIP(ctx, fl_spec_grad(s, n, P + i0 * n, n, C + i0 * n, n, W + i0 * n, n, op->logtheta,
                                     chunk_args(kind, alpha, sprm, i0, nb), dga + i0,
                                     kind == FL_SPEC_DIFFUSION ? dgs + i0 : nullptr));
    }
    if (GF) {
        FL_HIP(ctx, fl_scaled_gemm(s, n, op->V, op->ld, W, n, P, n, nb, nb, 1, Y, n));
        FL_HIP(ctx, fl_spmm_csr(s, n, op->rowptr, op->colidx, op->mval, nb, Y, n, GF, ldgf));
    }
    if (want_param) {
        if (ga) FL_HIP(ctx, hipMemcpyAsync(ga, dga, nb * 8, hipMemcpyDeviceToHost, s));
        if (gs) FL_HIP(ctx, hipMemcpyAsync(gs, dgs, nb * 8, hipMemcpyDeviceToHost, s));
        FL_HIP(ctx, hipStreamSynchronize(s));
    }
    (void)who;
    return FL_OK;
}

void destroy_graph(ApplyGraph* g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->ws) (void)hipFree(g->ws);
    delete g;
}

int ensure_graph_stream(fl_ctx* ctx) {
    if (ctx->graph_stream) return FL_OK;
    FL_HIP(ctx, hipStreamCreateWithFlags(&ctx->graph_stream, hipStreamNonBlocking));
    FL_HIP(ctx, hipEventCreateWithFlags(&ctx->graph_in, hipEventDisableTiming));
    FL_HIP(ctx, hipEventCreateWithFlags(&ctx->graph_out, hipEventDisableTiming));
    return FL_OK;
}

bool same_key(const ApplyGraph* g, const SpecCall& c) {
    if (g->kind != c.kind || g->nf != c.nf || g->ldf != c.ldf || g->na != c.na || g->ldu != c.ldu ||
        g->paired != c.paired || g->F != c.F || g->U != c.U)
        return false;
    if (std::memcmp(g->alpha.data(), c.alpha, sizeof(double) * c.na) != 0) return false;
    if (c.sprm && std::memcmp(g->sprm.data(), c.sprm, sizeof(double) * c.na) != 0) return false;
    return true;
}

}  // namespace

size_t fl_spectral_ws_doubles(int64_t n, int64_t nf, int64_t na) { return (size_t)n * (2 * nf + na); }

hipError_t fl_queue_spectral(const fl_op* op, hipStream_t s, const SpecCall& c, double* ws, const SplitWs* split,
                             bool timed) {
    const int64_t n = op->n;
    double* G = ws;
    double* C = G + (size_t)n * c.nf;
    double* W = C + (size_t)n * c.nf;
    hipError_t e;
    if ((e = fl_spmm_csr(s, n, op->rowptr, op->colidx, op->mval, c.nf, c.F, c.ldf, G, n)) != hipSuccess) return e;
    if (split)
        e = fl_dgemm_ws(s, 1, 0, n, c.nf, n, 1.0, op->V, op->ld, G, n, 0.0, C, n, split);
    else
        e = fl_dgemm(s, 1, 0, n, c.nf, n, 1.0, op->V, op->ld, G, n, 0.0, C, n);
    if (e != hipSuccess) return e;
    if ((e = queue_weights(op, s, c.kind, c.alpha, c.sprm, c.na, W)) != hipSuccess) return e;
    return fl_scaled_gemm(s, n, op->V, op->ld, W, n, C, n, c.nf, c.na, c.paired, c.U, c.ldu, nullptr, timed);
}

void fl_op_release_spectral(fl_op* op) {
    for (ApplyGraph* g : op->graphs) destroy_graph(g);
    op->graphs.clear();
    for (OpWs& w : op->ws)
        if (w.p) (void)hipFree(w.p);
    op->ws.clear();
}

extern "C" {

int fl_apply_fractional(fl_op* op, int64_t nf, const double* F, int64_t ldf, int64_t na, const double* alpha,
                        int paired, double* U, int64_t ldu) {
    if (!op) return FL_EINVAL;
    fl_ctx* ctx = op->ctx;
    const int64_t n = op->n;
    if (!op->has_eig) return fl_fail(ctx, FL_ESTATE, "fl_apply_fractional: eigensolve first");
    if (nf <= 0 || na <= 0 || !F || !U || !alpha || ldf < n || ldu < n)
        return fl_fail(ctx, FL_EINVAL, "fl_apply_fractional: bad sizes or null pointer");
    if (paired && nf != na) return fl_fail(ctx, FL_EINVAL, "fl_apply_fractional: paired requires nf == na");
    int rc = check_params(ctx, "fl_apply_fractional", na, alpha, nullptr, nullptr);
    if (rc || (rc = set_device(ctx))) return rc;
    double* ws = nullptr;
    if ((rc = op_ws(op, ctx->stream, fl_spectral_ws_doubles(n, nf, na) * 8, &ws))) return rc;
    SpecCall c{FL_SPEC_FRACTIONAL, nf, F, ldf, na, alpha, nullptr, paired, U, ldu};
    FL_HIP(ctx, fl_queue_spectral(op, ctx->stream, c, ws, nullptr, true));
    return FL_OK;
}

int fl_grad_apply(fl_op* op, int64_t nb, const double* F, int64_t ldf, const double* alpha, const double* GU,
                  int64_t ldgu, double* GF, int64_t ldgf, double* galpha) {
    if (!op) return FL_EINVAL;
    fl_ctx* ctx = op->ctx;
    const int64_t n = op->n;
    if (!op->has_eig) return fl_fail(ctx, FL_ESTATE, "fl_grad_apply: eigensolve first");
    if (nb <= 0 || !GU || !alpha || ldgu < n || (GF && ldgf < n) || (galpha && (!F || ldf < n)))
        return fl_fail(ctx, FL_EINVAL, "fl_grad_apply: bad sizes or null pointer");
    int rc = check_params(ctx, "fl_grad_apply", nb, alpha, nullptr, nullptr);
    if (rc || (rc = set_device(ctx))) return rc;
    return grad_spectral(op, "fl_grad_apply", FL_SPEC_FRACTIONAL, nb, F, ldf, alpha, nullptr, GU, ldgu, GF, ldgf,
                         galpha, nullptr);
}

int fl_apply_diffusion(fl_op* op, int64_t nf, const double* U0, int64_t ldu0, int64_t na, const double* alpha,
                       const double* t, const double* mu, int paired, double* U, int64_t ldu) {
    if (!op) return FL_EINVAL;
    fl_ctx* ctx = op->ctx;
    const int64_t n = op->n;
    if (!op->has_eig) return fl_fail(ctx, FL_ESTATE, "fl_apply_diffusion: eigensolve first");
    if (nf <= 0 || na <= 0 || !U0 || !U || !alpha || !t || !mu || ldu0 < n || ldu < n)
        return fl_fail(ctx, FL_EINVAL, "fl_apply_diffusion: bad sizes or null pointer");
    if (paired && nf != na) return fl_fail(ctx, FL_EINVAL, "fl_apply_diffusion: paired requires nf == na");
    int rc = check_params(ctx, "fl_apply_diffusion", na, alpha, t, mu);
    if (rc || (rc = set_device(ctx))) return rc;
    std::vector<double> sprm(na);
    for (int64_t i = 0; i < na; ++i) sprm[i] = mu[i] * t[i];
    double* ws = nullptr;
    if ((rc = op_ws(op, ctx->stream, fl_spectral_ws_doubles(n, nf, na) * 8, &ws))) return rc;
    SpecCall c{FL_SPEC_DIFFUSION, nf, U0, ldu0, na, alpha, sprm.data(), paired, U, ldu};
    FL_HIP(ctx, fl_queue_spectral(op, ctx->stream, c, ws, nullptr, true));
    return FL_OK;
}

int fl_grad_diffusion(fl_op* op, int64_t nb, const double* U0, int64_t ldu0, const double* alpha, const double* t,
                      const double* mu, const double* GU, int64_t ldgu, double* GU0, int64_t ldgu0, double* galpha,
                      double* gt, double* gmu) {
    if (!op) return FL_EINVAL;
    fl_ctx* ctx = op->ctx;
    const int64_t n = op->n;
    if (!op->has_eig) return fl_fail(ctx, FL_ESTATE, "fl_grad_diffusion: eigensolve first");
    const bool want_param = galpha || gt || gmu;
    if (nb <= 0 || !GU || !alpha || !t || !mu || ldgu < n || (GU0 && ldgu0 < n) ||
        (want_param && (!U0 || ldu0 < n)))
        return fl_fail(ctx, FL_EINVAL, "fl_grad_diffusion: bad sizes or null pointer");
    int rc = check_params(ctx, "fl_grad_diffusion", nb, alpha, t, mu);
    if (rc || (rc = set_device(ctx))) return rc;
    std::vector<double> sprm(nb), gs(nb, 0.0), ga(nb, 0.0);
    for (int64_t i = 0; i < nb; ++i) sprm[i] = mu[i] * t[i];
    rc = grad_spectral(op, "fl_grad_diffusion", FL_SPEC_DIFFUSION, nb, U0, ldu0, alpha, sprm.data(), GU, ldgu, GU0,
                       ldgu0, want_param ? ga.data() : nullptr, want_param ? gs.data() : nullptr);
    if (rc) return rc;
    // s = mu t: dL/dt = mu dL/ds, dL/dmu = t dL/ds
    for (int64_t i = 0; i < nb; ++i) {
        if (galpha) galpha[i] = ga[i];
        if (gt) gt[i] = mu[i] * gs[i];
        if (gmu) gmu[i] = t[i] * gs[i];
    }
    return FL_OK;
}

int fl_apply_graph(fl_op* op, int64_t nf, const double* F, int64_t ldf, int64_t na, const double* alpha, int paired,
                   double* U, int64_t ldu) {
    if (!op) return FL_EINVAL;
    fl_ctx* ctx = op->ctx;
    const int64_t n = op->n;
    if (!op->has_eig) return fl_fail(ctx, FL_ESTATE, "fl_apply_graph: eigensolve first");
    if (nf <= 0 || na <= 0 || !F || !U || !alpha || ldf < n || ldu < n)
        return fl_fail(ctx, FL_EINVAL, "fl_apply_graph: bad sizes or null pointer");
    if (paired && nf != na) return fl_fail(ctx, FL_EINVAL, "fl_apply_graph: paired requires nf == na");
    int rc = check_params(ctx, "fl_apply_graph", na, alpha, nullptr, nullptr);
    if (rc || (rc = set_device(ctx)) || (rc = ensure_graph_stream(ctx))) return rc;
    if (capturing(ctx->stream))
        return fl_fail(ctx, FL_ESTATE, "fl_apply_graph: the caller's stream is being captured");
    SpecCall c{FL_SPEC_FRACTIONAL, nf, F, ldf, na, alpha, nullptr, paired, U, ldu};
    hipStream_t gs = ctx->graph_stream;
    ApplyGraph* g = nullptr;
    for (ApplyGraph* x : op->graphs)
        if (same_key(x, c)) g = x;
    if (!g) {
        if (op->graphs.size() >= MAX_GRAPHS_PER_OP) {
            // evict the least recently replayed graph once its replays are done
            auto it = std::min_element(op->graphs.begin(), op->graphs.end(),
                                       [](const ApplyGraph* a, const ApplyGraph* b) { return a->last_use < b->last_use; });
            FL_HIP(ctx, hipStreamSynchronize(gs));
            destroy_graph(*it);
            op->graphs.erase(it);
        }
        g = new ApplyGraph();
        g->kind = c.kind;
        g->nf = nf;
        g->ldf = ldf;
        g->na = na;
        g->ldu = ldu;
        g->paired = paired;
        g->F = F;
        g->U = U;
        g->alpha.assign(alpha, alpha + na);
        void* p = nullptr;
        if (hipMalloc(&p, fl_spectral_ws_doubles(n, nf, na) * 8) != hipSuccess) {
            (void)hipGetLastError();
            delete g;
            return fl_fail(ctx, FL_ENOMEM, "fl_apply_graph: workspace allocation failed");
        }
        g->ws = static_cast<double*>(p);
        // the replay stream's split-k buffer exists before the capture starts
        (void)fl_stream_splitk_ws(gs);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t eq = fl_queue_spectral(op, gs, c, g->ws, nullptr, false);
            e = hipStreamEndCapture(gs, &graph);
            if (eq != hipSuccess) e = eq;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            destroy_graph(g);
            return fl_fail(ctx, FL_EHIP, std::string("fl_apply_graph: capture failed: ") + hipGetErrorString(e));
        }
        op->graphs.push_back(g);
    }
    g->last_use = ++op->graph_clock;
    FL_HIP(ctx, hipEventRecord(ctx->graph_in, ctx->stream));
    FL_HIP(ctx, hipStreamWaitEvent(gs, ctx->graph_in, 0));
    FL_HIP(ctx, hipGraphLaunch(g->exec, gs));
    FL_HIP(ctx, hipEventRecord(ctx->graph_out, gs));
    FL_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->graph_out, 0));
    return FL_OK;
}

}  // extern "C"
