// C-ABI of the fraclap library (declarations and contracts in fraclap.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>
#include "internal.h"

int fl_fail(fl_ctx* ctx, int code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return code;
}

namespace {

int set_device(fl_ctx* ctx) {
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fl_fail(ctx, FL_EHIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    return FL_OK;
}

template <class T>
int dev_alloc(fl_ctx* ctx, T** p, size_t count) {
    *p = nullptr;
    hipError_t e = hipMalloc((void**)p, sizeof(T) * (count > 0 ? count : 1));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fl_fail(ctx, FL_ENOMEM, "device allocation of " + std::to_string(sizeof(T) * count) + " bytes failed");
    }
    return FL_OK;
}

void dev_free(void* p) {
    if (p) (void)hipFree(p);
}

bool all_finite(const double* p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

int64_t pad_ld(int64_t n) { return ((n + 15) / 16) * 16; }

// Build the CSR pattern of the Galerkin matrices from element connectivity.
void csr_from_elements(int64_t n, int nv, int64_t n_elem, const int32_t* conn, const std::vector<int64_t>& dof,
                       std::vector<int32_t>& rowptr, std::vector<int32_t>& colidx) {
    std::vector<std::vector<int32_t>> rows(n);
    for (int64_t e = 0; e < n_elem; ++e)
        for (int a = 0; a < nv; ++a) {
            int64_t i = dof[conn[e * nv + a]];
            if (i < 0) continue;
            for (int b = 0; b < nv; ++b) {
                int64_t j = dof[conn[e * nv + b]];
                if (j >= 0) rows[i].push_back((int32_t)j);
            }
        }
    rowptr.assign(n + 1, 0);
    colidx.clear();
    for (int64_t i = 0; i < n; ++i) {
        auto& r = rows[i];
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        colidx.insert(colidx.end(), r.begin(), r.end());
        rowptr[i + 1] = (int32_t)colidx.size();
    }
}

int upload_csr_and_gather(fl_op* op, const std::vector<int32_t>& rowptr, const std::vector<int32_t>& colidx) {
    fl_ctx* ctx = op->ctx;
    op->nnz = (int64_t)colidx.size();
    int rc;
    if ((rc = dev_alloc(ctx, &op->rowptr, rowptr.size())) || (rc = dev_alloc(ctx, &op->colidx, colidx.size())) ||
        (rc = dev_alloc(ctx, &op->kval, colidx.size())) || (rc = dev_alloc(ctx, &op->mval, colidx.size())))
        return rc;
    FL_HIP(ctx, hipMemcpyAsync(op->rowptr, rowptr.data(), rowptr.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    FL_HIP(ctx, hipMemcpyAsync(op->colidx, colidx.data(), colidx.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    FL_HIP(ctx, fl_csr_gather(ctx->stream, op->n, op->rowptr, op->colidx, op->K, op->M, op->ld, op->kval, op->mval));
    return FL_OK;
}

}  // namespace

// K := L^-1 K L^-T given L and the inverses of its 128 x 128 diagonal blocks.
int fl_sygst_device(fl_ctx* ctx, int64_t n, const double* L, int64_t ldl, const double* Linv, double* K,
                    int64_t ldk, double* work) {
    hipStream_t s = ctx->stream;
    FL_HIP(ctx, fl_trsm_lln(s, n, n, L, ldl, Linv, K, ldk, work));
    FL_HIP(ctx, fl_trsm_rlt(s, n, n, L, ldl, Linv, K, ldk, work));
    FL_HIP(ctx, fl_symmetrize(s, n, K, ldk));
    return FL_OK;
}

extern "C" {

int fl_ctx_create(int device, void* hip_stream, fl_ctx** out) {
    if (!out) return FL_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return FL_EINVAL;
    fl_ctx* c = new fl_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (set_device(c)) {
        delete c;
        return FL_EHIP;
    }
    *out = c;
    return FL_OK;
}

int fl_ctx_set_stream(fl_ctx* ctx, void* hip_stream) {
    if (!ctx) return FL_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    return FL_OK;
}

void fl_ctx_destroy(fl_ctx* ctx) {
    if (!ctx) return;
    if (ctx->graph_stream) {
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(ctx->graph_stream);
        (void)hipStreamDestroy(ctx->graph_stream);
    }
    if (ctx->graph_in) (void)hipEventDestroy(ctx->graph_in);
    if (ctx->graph_out) (void)hipEventDestroy(ctx->graph_out);
    delete ctx;
}

const char* fl_last_error(const fl_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int64_t fl_op_n(const fl_op* op) { return op ? op->n : -1; }

void fl_op_destroy(fl_op* op) {
    if (!op) return;
    (void)hipSetDevice(op->device);
    (void)hipDeviceSynchronize();
    dev_free(op->K);
    dev_free(op->M);
    dev_free(op->rowptr);
    dev_free(op->colidx);
    dev_free(op->kval);
    dev_free(op->mval);
    dev_free(op->theta);
    dev_free(op->logtheta);
    dev_free(op->V);
    dev_free(op->inert_pinv);
    fl_op_release_spectral(op);
    delete op;
}

}  // extern "C"

// Assembly into dense K and M plus their CSR copies (dense = true), or into
// the CSR values only (dense = false: pencils too large for dense storage).
static int assemble_impl(fl_ctx* ctx, bool dense, int elem, int64_t n_nodes, const double* xy, int64_t n_elem,
                         const int32_t* conn, const uint8_t* dirichlet, fl_op** out, int64_t* n_dof,
                         int64_t* dof_of_node) {
    if (!ctx) return FL_EINVAL;
    if (!out || !xy || !conn || !dirichlet || n_nodes <= 0 || n_elem <= 0)
        return fl_fail(ctx, FL_EINVAL, "fl_assemble: null pointer or empty mesh");
    *out = nullptr;
    int order = 0;  // tensor-product order for elem = (p + 1)^2 > 4
    if (elem != FL_ELEM_Q1 && elem != FL_ELEM_P1) {
        for (int p = 2; p <= 8; ++p)
            if (elem == (p + 1) * (p + 1)) order = p;
        if (!order) return fl_fail(ctx, FL_EINVAL, "fl_assemble: elem must be 3, 4 or (p+1)^2 with 2 <= p <= 8");
    }
    if (!all_finite(xy, (size_t)n_nodes * 2)) return fl_fail(ctx, FL_EINVAL, "fl_assemble: non-finite coordinate");
    const int nv = elem;
    // validate elements
    for (int64_t e = 0; e < n_elem; ++e) {
        double x[81], y[81];
        for (int a = 0; a < nv; ++a) {
            int32_t v = conn[e * nv + a];
            if (v < 0 || v >= n_nodes)
                return fl_fail(ctx, FL_EINVAL, "fl_assemble: element " + std::to_string(e) + " has node out of range");
            x[a] = xy[2 * (int64_t)v];
            y[a] = xy[2 * (int64_t)v + 1];
        }
        if (nv == 3) {
            double det = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
            if (!(det > 0.0))
                return fl_fail(ctx, FL_EINVAL, "fl_assemble: triangle " + std::to_string(e) + " is clockwise or degenerate");
        } else if (nv == 4) {
            double xmin = std::min(std::min(x[0], x[1]), std::min(x[2], x[3]));
            double xmax = std::max(std::max(x[0], x[1]), std::max(x[2], x[3]));
            double ymin = std::min(std::min(y[0], y[1]), std::min(y[2], y[3]));
            double ymax = std::max(std::max(y[0], y[1]), std::max(y[2], y[3]));
            bool ok = xmax > xmin && ymax > ymin;
            int seen = 0;
            for (int a = 0; a < 4 && ok; ++a) {
                bool ex = (x[a] == xmin || x[a] == xmax), ey = (y[a] == ymin || y[a] == ymax);
                if (!ex || !ey) ok = false;
                seen |= 1 << ((x[a] == xmax ? 1 : 0) + 2 * (y[a] == ymax ? 1 : 0));
            }
            // counter-clockwise: signed area of the polygon positive
            double sa = 0.0;
            for (int a = 0; a < 4; ++a) sa += x[a] * y[(a + 1) % 4] - x[(a + 1) % 4] * y[a];
            if (!ok || seen != 15 || !(sa > 0.0))
                return fl_fail(ctx, FL_EINVAL,
                               "fl_assemble: quadrilateral " + std::to_string(e) +
                                   " is not a counter-clockwise axis-aligned rectangle");
        } else {
            // tensor lattice: node (a, b) at (x of (a, 0), y of (0, b)), both increasing
            const int q = order + 1;
            bool ok = true;
            for (int b = 0; b < q && ok; ++b)
                for (int a = 0; a < q && ok; ++a) {
                    const int i = a + q * b;
                    if (x[i] != x[a] || y[i] != y[q * b]) ok = false;
                    if (a > 0 && !(x[a] > x[a - 1])) ok = false;
                    if (b > 0 && !(y[q * b] > y[q * (b - 1)])) ok = false;
                }
            if (!ok)
                return fl_fail(ctx, FL_EINVAL,
                               "fl_assemble: order-" + std::to_string(order) + " element " + std::to_string(e) +
                                   " is not an increasing tensor lattice on an axis-aligned rectangle");
        }
    }
    std::vector<int64_t> dof(n_nodes, -1);
    int64_t n = 0;
    for (int64_t v = 0; v < n_nodes; ++v)
        if (!dirichlet[v]) dof[v] = n++;
    if (n == 0) return fl_fail(ctx, FL_EINVAL, "fl_assemble: no interior node");
    if (n_dof) *n_dof = n;
    if (dof_of_node) std::memcpy(dof_of_node, dof.data(), sizeof(int64_t) * n_nodes);
    // greedy element colouring: no two elements of a colour share a node
    std::vector<uint64_t> used(n_nodes, 0);
    std::vector<int> color(n_elem, 0);
    int ncolor = 0;
    for (int64_t e = 0; e < n_elem; ++e) {
        uint64_t busy = 0;
        for (int a = 0; a < nv; ++a) busy |= used[conn[e * nv + a]];
        int c = 0;
        while (c < 64 && (busy >> c & 1ull)) ++c;
        if (c == 64) return fl_fail(ctx, FL_EINVAL, "fl_assemble: more than 64 element colours needed");
        color[e] = c;
        ncolor = std::max(ncolor, c + 1);
        for (int a = 0; a < nv; ++a) used[conn[e * nv + a]] |= 1ull << c;
    }
    std::vector<int64_t> cstart(ncolor + 1, 0);
    for (int64_t e = 0; e < n_elem; ++e) cstart[color[e] + 1]++;
    for (int c = 0; c < ncolor; ++c) cstart[c + 1] += cstart[c];
    std::vector<int32_t> sorted((size_t)n_elem * nv);
    {
        std::vector<int64_t> pos(cstart.begin(), cstart.end() - 1);
        for (int64_t e = 0; e < n_elem; ++e) {
            int64_t p = pos[color[e]]++;
            std::memcpy(&sorted[p * nv], &conn[e * nv], sizeof(int32_t) * nv);
        }
    }
    std::vector<int32_t> rowptr, colidx;
    csr_from_elements(n, nv, n_elem, conn, dof, rowptr, colidx);

    int rc = set_device(ctx);
    if (rc) return rc;
    fl_op* op = new fl_op();
    op->ctx = ctx;
    op->device = ctx->device;
    op->n = n;
    op->ld = pad_ld(n);
    size_t nn = (size_t)op->ld * n;
    double* dxy = nullptr;
    int32_t* dconn = nullptr;
    int64_t* ddof = nullptr;
    auto cleanup = [&]() {
        dev_free(dxy);
        dev_free(dconn);
        dev_free(ddof);
    };
    if ((dense && ((rc = dev_alloc(ctx, &op->K, nn)) || (rc = dev_alloc(ctx, &op->M, nn)))) ||
        (rc = dev_alloc(ctx, &dxy, (size_t)n_nodes * 2)) || (rc = dev_alloc(ctx, &dconn, sorted.size())) ||
        (rc = dev_alloc(ctx, &ddof, (size_t)n_nodes))) {
        cleanup();
        fl_op_destroy(op);
        return rc;
    }
    hipStream_t s = ctx->stream;
    hipError_t he = hipSuccess;
    if ((he = hipMemcpyAsync(dxy, xy, (size_t)n_nodes * 16, hipMemcpyHostToDevice, s)) ||
        (he = hipMemcpyAsync(dconn, sorted.data(), sorted.size() * 4, hipMemcpyHostToDevice, s)) ||
        (he = hipMemcpyAsync(ddof, dof.data(), (size_t)n_nodes * 8, hipMemcpyHostToDevice, s))) {
        cleanup();
        fl_op_destroy(op);
        return fl_fail(ctx, FL_EHIP, std::string("fl_assemble: ") + hipGetErrorString(he));
    }
    if (dense) {
        if ((he = hipMemsetAsync(op->K, 0, nn * 8, s)) || (he = hipMemsetAsync(op->M, 0, nn * 8, s)) ||
            (he = fl_assemble_launch(s, elem, dxy, dconn, cstart.data(), ncolor, ddof, n, op->ld, op->K, op->M)) ||
            (he = hipStreamSynchronize(s))) {
            cleanup();
            fl_op_destroy(op);
            return fl_fail(ctx, FL_EHIP, std::string("fl_assemble: ") + hipGetErrorString(he));
        }
        cleanup();
        rc = upload_csr_and_gather(op, rowptr, colidx);
    } else {
        // the pattern first, then the element contributions straight into its values
        op->nnz = (int64_t)colidx.size();
        if (!(rc = dev_alloc(ctx, &op->rowptr, rowptr.size())) && !(rc = dev_alloc(ctx, &op->colidx, colidx.size())) &&
            !(rc = dev_alloc(ctx, &op->kval, colidx.size())) && !(rc = dev_alloc(ctx, &op->mval, colidx.size()))) {
            if ((he = hipMemcpyAsync(op->rowptr, rowptr.data(), rowptr.size() * 4, hipMemcpyHostToDevice, s)) ||
                (he = hipMemcpyAsync(op->colidx, colidx.data(), colidx.size() * 4, hipMemcpyHostToDevice, s)) ||
                (he = hipMemsetAsync(op->kval, 0, colidx.size() * 8, s)) ||
                (he = hipMemsetAsync(op->mval, 0, colidx.size() * 8, s)) ||
                (he = fl_assemble_csr_launch(s, elem, dxy, dconn, cstart.data(), ncolor, ddof, op->rowptr, op->colidx,
                                             op->kval, op->mval)))
                rc = fl_fail(ctx, FL_EHIP, std::string("fl_assemble_sparse: ") + hipGetErrorString(he));
        }
        if (!rc && (he = hipStreamSynchronize(s)) != hipSuccess)
            rc = fl_fail(ctx, FL_EHIP, std::string("fl_assemble_sparse: ") + hipGetErrorString(he));
        cleanup();
    }
    if (!rc) {
        he = hipStreamSynchronize(s);
        if (he != hipSuccess) rc = fl_fail(ctx, FL_EHIP, std::string("fl_assemble: ") + hipGetErrorString(he));
    }
    if (rc) {
        fl_op_destroy(op);
        return rc;
    }
    *out = op;
    return FL_OK;
}

extern "C" {

int fl_assemble(fl_ctx* ctx, int elem, int64_t n_nodes, const double* xy, int64_t n_elem, const int32_t* conn,
                const uint8_t* dirichlet, fl_op** out, int64_t* n_dof, int64_t* dof_of_node) {
    return assemble_impl(ctx, true, elem, n_nodes, xy, n_elem, conn, dirichlet, out, n_dof, dof_of_node);
}

int fl_assemble_sparse(fl_ctx* ctx, int elem, int64_t n_nodes, const double* xy, int64_t n_elem, const int32_t* conn,
                       const uint8_t* dirichlet, fl_op** out, int64_t* n_dof, int64_t* dof_of_node) {
    return assemble_impl(ctx, false, elem, n_nodes, xy, n_elem, conn, dirichlet, out, n_dof, dof_of_node);
}

int fl_op_from_dense(fl_ctx* ctx, int64_t n, const double* K, const double* M, int64_t ld, int on_device,
                     fl_op** out) {
    if (!ctx) return FL_EINVAL;
    if (!out || !K || !M || n <= 0 || ld < n) return fl_fail(ctx, FL_EINVAL, "fl_op_from_dense: bad arguments");
    *out = nullptr;
    int rc = set_device(ctx);
    if (rc) return rc;
    // host copies (validation and the CSR pattern are built on the host)
    std::vector<double> hk((size_t)n * n), hm((size_t)n * n);
    hipStream_t s = ctx->stream;
    if (on_device) {
        FL_HIP(ctx, hipMemcpy2DAsync(hk.data(), n * 8, K, ld * 8, n * 8, n, hipMemcpyDeviceToHost, s));
        FL_HIP(ctx, hipMemcpy2DAsync(hm.data(), n * 8, M, ld * 8, n * 8, n, hipMemcpyDeviceToHost, s));
        FL_HIP(ctx, hipStreamSynchronize(s));
    } else {
        for (int64_t j = 0; j < n; ++j) {
            std::memcpy(&hk[j * n], K + j * ld, n * 8);
            std::memcpy(&hm[j * n], M + j * ld, n * 8);
        }
    }
    if (!all_finite(hk.data(), hk.size()) || !all_finite(hm.data(), hm.size()))
        return fl_fail(ctx, FL_EINVAL, "fl_op_from_dense: non-finite entry");
    std::vector<int32_t> rowptr(n + 1, 0), colidx;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j)
            if (hk[i + j * n] != 0.0 || hm[i + j * n] != 0.0) colidx.push_back((int32_t)j);
        rowptr[i + 1] = (int32_t)colidx.size();
    }
    fl_op* op = new fl_op();
    op->ctx = ctx;
    op->device = ctx->device;
    op->n = n;
    op->ld = pad_ld(n);
    size_t nn = (size_t)op->ld * n;
    if ((rc = dev_alloc(ctx, &op->K, nn)) || (rc = dev_alloc(ctx, &op->M, nn))) {
        fl_op_destroy(op);
        return rc;
    }
    hipError_t he;
    if ((he = hipMemcpy2DAsync(op->K, op->ld * 8, hk.data(), n * 8, n * 8, n, hipMemcpyHostToDevice, s)) ||
        (he = hipMemcpy2DAsync(op->M, op->ld * 8, hm.data(), n * 8, n * 8, n, hipMemcpyHostToDevice, s))) {
        fl_op_destroy(op);
        return fl_fail(ctx, FL_EHIP, hipGetErrorString(he));
    }
    rc = upload_csr_and_gather(op, rowptr, colidx);
    if (!rc && (he = hipStreamSynchronize(s)) != hipSuccess) rc = fl_fail(ctx, FL_EHIP, hipGetErrorString(he));
    if (rc) {
        fl_op_destroy(op);
        return rc;
    }
    *out = op;
    return FL_OK;
}

int fl_op_matrices(const fl_op* op, double* K, double* M, int64_t ld, int on_device) {
    if (!op) return FL_EINVAL;
    fl_ctx* ctx = op->ctx;
    if (!op->K || !op->M) return fl_fail(ctx, FL_ESTATE, "fl_op_matrices: the operator holds no dense pencil");
    if (ld < op->n) return fl_fail(ctx, FL_EINVAL, "fl_op_matrices: ld < n");
    int rc = set_device(ctx);
    if (rc) return rc;
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    int64_t n = op->n;
    if (K) FL_HIP(ctx, hipMemcpy2DAsync(K, ld * 8, op->K, op->ld * 8, n * 8, n, kind, ctx->stream));
    if (M) FL_HIP(ctx, hipMemcpy2DAsync(M, ld * 8, op->M, op->ld * 8, n * 8, n, kind, ctx->stream));
    FL_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return FL_OK;
}

static int alloc_eig(fl_op* op) {
    int rc;
    if (!op->theta && (rc = dev_alloc(op->ctx, &op->theta, op->n))) return rc;
    if (!op->logtheta && (rc = dev_alloc(op->ctx, &op->logtheta, op->n))) return rc;
    if (!op->V && (rc = dev_alloc(op->ctx, &op->V, (size_t)op->ld * op->n))) return rc;
    return FL_OK;
}

int fl_op_set_eigenpairs(fl_op* op, const double* theta, const double* V, int64_t ldv, int on_device) {
    if (!op) return FL_EINVAL;
    fl_ctx* ctx = op->ctx;
    if (!theta || !V || ldv < op->n) return fl_fail(ctx, FL_EINVAL, "fl_op_set_eigenpairs: bad arguments");
    int rc = set_device(ctx);
    if (rc) return rc;
    int64_t n = op->n;
    std::vector<double> th(n);
    if (on_device) {
        FL_HIP(ctx, hipMemcpy(th.data(), theta, n * 8, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(th.data(), theta, n * 8);
    }
    for (double t : th)
        if (!(t > 0.0) || !std::isfinite(t))
            return fl_fail(ctx, FL_EINVAL, "fl_op_set_eigenpairs: eigenvalues must be positive and finite");
    if ((rc = alloc_eig(op))) return rc;
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    FL_HIP(ctx, hipMemcpyAsync(op->theta, th.data(), n * 8, hipMemcpyHostToDevice, ctx->stream));
    FL_HIP(ctx, hipMemcpy2DAsync(op->V, op->ld * 8, V, ldv * 8, n * 8, n, kind, ctx->stream));
    FL_HIP(ctx, fl_log_kernel(ctx->stream, n, op->theta, op->logtheta));
    FL_HIP(ctx, hipStreamSynchronize(ctx->stream));
    op->has_eig = 1;
    op->eig_precision = -1;
    op->refine_iters = 0;
    op->refine_resid = 0.0;
    return FL_OK;
}

int fl_eigenpairs(const fl_op* op, double* theta, double* V, int64_t ldv, int on_device) {
    if (!op) return FL_EINVAL;
    fl_ctx* ctx = op->ctx;
    if (!op->has_eig) return fl_fail(ctx, FL_ESTATE, "fl_eigenpairs: no eigenpairs yet");
    if (V && ldv < op->n) return fl_fail(ctx, FL_EINVAL, "fl_eigenpairs: ldv < n");
    int rc = set_device(ctx);
    if (rc) return rc;
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (theta) FL_HIP(ctx, hipMemcpyAsync(theta, op->theta, op->n * 8, kind, ctx->stream));
    if (V) FL_HIP(ctx, hipMemcpy2DAsync(V, ldv * 8, op->V, op->ld * 8, op->n * 8, op->n, kind, ctx->stream));
    FL_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return FL_OK;
}

// ------------------------------------------------------------ stage calls
int fl_dgemm(fl_ctx* ctx, int ta, int tb, int64_t m, int64_t n, int64_t k, double alpha, const double* A,
             int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc) {
    if (!ctx) return FL_EINVAL;
    if (m < 0 || n < 0 || k < 0 || ldc < std::max<int64_t>(1, m) ||
        lda < std::max<int64_t>(1, ta ? k : m) || ldb < std::max<int64_t>(1, tb ? n : k))
        return fl_fail(ctx, FL_EINVAL, "fl_dgemm: bad sizes");
    int rc = set_device(ctx);
    if (rc) return rc;
    FL_HIP(ctx, ::fl_dgemm(ctx->stream, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc));
    FL_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return FL_OK;
}

int fl_dpotrf(fl_ctx* ctx, int64_t n, double* A, int64_t lda, int64_t* info) {
    if (!ctx) return FL_EINVAL;
    if (n <= 0 || lda < n || !A) return fl_fail(ctx, FL_EINVAL, "fl_dpotrf: bad arguments");
    int rc = set_device(ctx);
    if (rc) return rc;
    DevBuf linv, work, dinfo;
    FL_HIP(ctx, linv.alloc(sizeof(double) * fl_potrf_linv_elems(n)));
    FL_HIP(ctx, work.alloc(sizeof(double) * fl_trsm_work_elems(n, n)));
    FL_HIP(ctx, dinfo.alloc(sizeof(int64_t)));
    FL_HIP(ctx, hipMemsetAsync(dinfo.p, 0, 8, ctx->stream));
    FL_HIP(ctx, fl_potrf(ctx->stream, n, A, lda, linv.as<double>(), dinfo.as<int64_t>(), work.as<double>()));
    int64_t h = 0;
    FL_HIP(ctx, hipMemcpyAsync(&h, dinfo.p, 8, hipMemcpyDeviceToHost, ctx->stream));
    FL_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (info) *info = h;
    if (h) return fl_fail(ctx, FL_ENOTSPD, "fl_dpotrf: not positive definite at pivot " + std::to_string(h));
    return FL_OK;
}

int fl_dsygst(fl_ctx* ctx, int64_t n, const double* L, int64_t ldl, double* K, int64_t ldk) {
    if (!ctx) return FL_EINVAL;
    if (n <= 0 || ldl < n || ldk < n || !L || !K) return fl_fail(ctx, FL_EINVAL, "fl_dsygst: bad arguments");
    int rc = set_device(ctx);
    if (rc) return rc;
    DevBuf linv, work;
    FL_HIP(ctx, linv.alloc(sizeof(double) * fl_potrf_linv_elems(n)));
    FL_HIP(ctx, work.alloc(sizeof(double) * fl_trsm_work_elems(n, n)));
    FL_HIP(ctx, fl_trtri_leaves(ctx->stream, n, L, ldl, linv.as<double>()));
    rc = fl_sygst_device(ctx, n, L, ldl, linv.as<double>(), K, ldk, work.as<double>());
    if (rc) return rc;
    FL_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return FL_OK;
}

}  // extern "C"
