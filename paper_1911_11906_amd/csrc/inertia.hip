// Eigenvalue counting by Sylvester's law of inertia (Section "Eigenvalue
// counting"): the number of eigenvalues of K phi = theta M phi below sigma
// equals the number of negative pivots of an LDL^T factorisation of
// K - sigma M.  A symmetric permutation is a congruence and keeps the
// inertia, so the pencil is first reordered to a small bandwidth (the
// natural numbering or reverse Cuthill-McKee, whichever is narrower; FEM
// pencils of n unknowns have a bandwidth near sqrt(n)), and each shift's
// banded matrix is factored without pivoting.
//
// One workgroup per shift.  The band of K - sigma M lives in device memory
// (lower band, column-major, (bw + 1) rows); the factorisation runs in
// blocks of NB columns: the block's panel (its columns, bw + NB rows) is
// staged in LDS and factored there (right-looking, one barrier per column,
// columns kept unscaled: P[r][c] = l_rc d_c), then the panel's rank-NB
// update is applied to the band of the next bw columns in device memory
// (each entry's NB-term sum read from LDS).  Only the signs of the pivots are
// kept (or, for the solves of spectrum slicing, the whole factor).  An
// exactly zero pivot makes the count for that shift -1.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <queue>
#include <string>
#include <vector>
#include "internal.h"

namespace {

constexpr int INB = 32;     // columns per block
constexpr int INT = 256;    // threads per workgroup
constexpr int IBWMAX = FL_BAND_MAX; // largest bandwidth (panel rows bw + NB fit in LDS)
constexpr int IPR = IBWMAX + INB + 1;  // LDS row stride of the panel

// The band of K - sigma_s M for every shift s (scattered from the CSR
// pencil through the permutation; the band must be zero on entry).
__global__ void band_build_kernel(int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                                  const double* __restrict__ kval, const double* __restrict__ mval,
                                  const int32_t* __restrict__ pinv, const double* __restrict__ sigma, int64_t ldb,
                                  int64_t stride, double* band) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double sg = sigma[blockIdx.y];
    double* B = band + (int64_t)blockIdx.y * stride;
    const int64_t pi = pinv[i];
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        const int64_t pj = pinv[colidx[p]];
        if (pi >= pj) B[(pi - pj) + pj * ldb] = kval[p] - sg * mval[p];
    }
}

// Workgroup barrier that also orders the workgroup's device-memory traffic:
// every wave drains its stores, then the vector L1 is invalidated so later
// loads see what the other waves wrote.
__device__ inline void wg_mem_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// STORE: the factor is kept for solves: the band (column layout) receives
// L below the diagonal and D on it, and Lrow (row layout, element (r, c) at
// (bw - (r - c)) + r ldb) the same entries by rows.
template <bool STORE>
__global__ __launch_bounds__(INT) void ldl_kernel(int64_t n, int bw, int64_t ldb, int64_t stride, double* band,
                                                  double* lrow, int64_t* counts) {
    __shared__ double P[IPR * INB];
    __shared__ double inv_d[INB];
    __shared__ int neg_s, zero_s;
    double* B = band + (int64_t)blockIdx.x * stride;
    double* R = STORE ? lrow + (int64_t)blockIdx.x * stride : nullptr;
    const int t = threadIdx.x;
    if (t == 0) {
        neg_s = 0;
        zero_s = 0;
    }
    for (int64_t j0 = 0; j0 < n; j0 += INB) {
        const int jb = (int)std::min<int64_t>(INB, n - j0);
        const int rows = (int)std::min<int64_t>(bw + jb, n - j0);
        // ---- panel: P[r][c] = A(j0 + r, j0 + c) inside the band, else 0
        for (int e = t; e < rows * jb; e += INT) {
            const int r = e % rows, c = e / rows;
            P[r + c * IPR] = (r >= c && r - c <= bw) ? B[(r - c) + (j0 + c) * ldb] : 0.0;
        }
        __syncthreads();
        // ---- factor the panel column by column
        for (int c = 0; c < jb; ++c) {
            const double d = P[c + c * IPR];
            if (d == 0.0) {
                if (t == 0) zero_s = 1;
                break;
            }
            if (t == 0) {
                if (d < 0.0) ++neg_s;
                inv_d[c] = 1.0 / d;
            }
            const int rlast = std::min(rows - 1, c + bw);  // last row of column c inside the band
            const int ncol = jb - 1 - c;                      // columns c + 1 .. jb - 1
            const int nr = rlast - c;                         // rows c + 1 .. rlast
            for (int e = t; e < ncol * nr; e += INT) {
                const int r = c + 1 + e % nr, cc = c + 1 + e / nr;
                if (r >= cc) P[r + cc * IPR] -= P[r + c * IPR] * P[cc + c * IPR] / d;
            }
            __syncthreads();
        }
        __syncthreads();
        if (zero_s) break;
        if (STORE) {
            // the block's columns of L and D, in both layouts
            for (int e = t; e < rows * jb; e += INT) {
                const int r = e % rows, c = e / rows;
                if (r < c || r - c > bw) continue;
                const double v = (r == c) ? P[c + c * IPR] : P[r + c * IPR] * inv_d[c];
                B[(r - c) + (j0 + c) * ldb] = v;
                R[(bw - (r - c)) + (j0 + r) * ldb] = v;
            }
        }
        // ---- rank-jb update of the next bw columns: A(r, q) -= sum_c P[r][c] P[q][c] / d_c
        // for q_l in [jb, jb + bw), r_l in [q_l, min(jb - 1 + bw, n - 1 - j0)]
        const int qn = (int)std::min<int64_t>(bw, n - j0 - jb);
        const int rmax = std::min(jb - 1 + bw, (int)(n - 1 - j0));
        const int nrr = rmax - jb + 1;  // candidate rows jb .. rmax
        for (int e = t; e < qn * nrr; e += INT) {
            const int r = jb + e % nrr, q = jb + e / nrr;
            if (r < q) continue;
            double s = 0.0;
            for (int c = 0; c < jb; ++c) s += P[r + c * IPR] * P[q + c * IPR] * inv_d[c];
            if (s != 0.0) B[(r - q) + (j0 + q) * ldb] -= s;
        }
        wg_mem_sync();
    }
    __syncthreads();
    if (t == 0) counts[blockIdx.x] = zero_s ? -1 : (int64_t)neg_s;
}

// Bandwidth of the pattern under the numbering new = pinv[old].
int64_t bandwidth(int64_t n, const std::vector<int32_t>& rowptr, const std::vector<int32_t>& colidx,
                  const std::vector<int32_t>& pinv) {
    int64_t bw = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            bw = std::max<int64_t>(bw, std::abs((int64_t)pinv[i] - (int64_t)pinv[colidx[p]]));
    return bw;
}

// Reverse Cuthill-McKee numbering (Cuthill and McKee 1969; reversed as
// proposed by George): breadth-first from a pseudo-peripheral start (the
// farthest node of repeated searches), neighbours visited by increasing
// degree, the order reversed.  Every connected component in turn.
std::vector<int32_t> rcm_pinv(int64_t n, const std::vector<int32_t>& rowptr, const std::vector<int32_t>& colidx) {
    std::vector<int32_t> deg(n), level(n), order;
    order.reserve(n);
    for (int64_t i = 0; i < n; ++i) deg[i] = rowptr[i + 1] - rowptr[i];
    std::vector<char> done(n, 0);
    auto bfs_last = [&](int32_t s) {  // last node reached (an eccentric one) and its depth
        std::fill(level.begin(), level.end(), -1);
        std::queue<int32_t> q;
        q.push(s);
        level[s] = 0;
        int32_t last = s;
        while (!q.empty()) {
            int32_t u = q.front();
            q.pop();
            last = u;
            for (int32_t p = rowptr[u]; p < rowptr[u + 1]; ++p) {
                int32_t v = colidx[p];
                if (level[v] < 0 && !done[v]) {
                    level[v] = level[u] + 1;
                    q.push(v);
                }
            }
        }
        return std::make_pair(last, level[last]);
    };
    for (int64_t seed = 0; seed < n; ++seed) {
        if (done[seed]) continue;
        // pseudo-peripheral node: hop to the farthest node while the depth grows
        int32_t s = (int32_t)seed;
        auto cur = bfs_last(s);
        for (int it = 0; it < 8; ++it) {
            auto nxt = bfs_last(cur.first);
            if (nxt.second <= cur.second) break;
            s = cur.first;
            cur = nxt;
        }
        s = cur.first;
        std::queue<int32_t> q;
        q.push(s);
        done[s] = 1;
        std::vector<int32_t> nb;
        while (!q.empty()) {
            int32_t u = q.front();
            q.pop();
            order.push_back(u);
            nb.clear();
            for (int32_t p = rowptr[u]; p < rowptr[u + 1]; ++p)
                if (!done[colidx[p]]) {
                    nb.push_back(colidx[p]);
                    done[colidx[p]] = 1;
                }
            std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) { return deg[a] < deg[b] || (deg[a] == deg[b] && a < b); });
            for (int32_t v : nb) q.push(v);
        }
    }
    std::vector<int32_t> pinv(n);
    for (int64_t k = 0; k < n; ++k) pinv[order[k]] = (int32_t)(n - 1 - k);
    return pinv;
}

// Numbering of the op's pattern with the smaller bandwidth (cached).
int prepare_ordering(fl_op* op);

}  // namespace

int fl_pattern_bandwidth(fl_op* op, int64_t* bw) {
    *bw = -1;
    if (!op->rowptr || !op->colidx) return FL_OK;
    if (op->natural_bw < 0) {
        const int64_t n = op->n;
        std::vector<int32_t> rowptr(n + 1), colidx(op->nnz);
        FL_HIP(op->ctx, hipMemcpy(rowptr.data(), op->rowptr, 4 * (n + 1), hipMemcpyDeviceToHost));
        FL_HIP(op->ctx, hipMemcpy(colidx.data(), op->colidx, 4 * op->nnz, hipMemcpyDeviceToHost));
        int64_t b = 0;
        for (int64_t i = 0; i < n; ++i)
            for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) b = std::max<int64_t>(b, std::abs(i - (int64_t)colidx[p]));
        op->natural_bw = b;
    }
    *bw = op->natural_bw;
    return FL_OK;
}

namespace {

int prepare_ordering(fl_op* op) {
    fl_ctx* ctx = op->ctx;
    if (op->inert_pinv) return FL_OK;
    const int64_t n = op->n;
    std::vector<int32_t> rowptr(n + 1), colidx(op->nnz);
    FL_HIP(ctx, hipMemcpy(rowptr.data(), op->rowptr, 4 * (n + 1), hipMemcpyDeviceToHost));
    FL_HIP(ctx, hipMemcpy(colidx.data(), op->colidx, 4 * op->nnz, hipMemcpyDeviceToHost));
    std::vector<int32_t> ident(n);
    for (int64_t i = 0; i < n; ++i) ident[i] = (int32_t)i;
    const int64_t bw0 = bandwidth(n, rowptr, colidx, ident);
    std::vector<int32_t> rcm = rcm_pinv(n, rowptr, colidx);
    const int64_t bw1 = bandwidth(n, rowptr, colidx, rcm);
    const std::vector<int32_t>& pick = bw1 < bw0 ? rcm : ident;
    op->inert_bw = std::min(bw0, bw1);
    void* p = nullptr;
    if (hipMalloc(&p, 4 * n) != hipSuccess) {
        (void)hipGetLastError();
        return fl_fail(ctx, FL_ENOMEM, "fl_inertia_count: allocation of the ordering failed");
    }
    op->inert_pinv = static_cast<int32_t*>(p);
    FL_HIP(ctx, hipMemcpy(op->inert_pinv, pick.data(), 4 * n, hipMemcpyHostToDevice));
    return FL_OK;
}

}  // namespace

int fl_inertia_prepare(fl_op* op) { return prepare_ordering(op); }

int64_t fl_band_ldb(int64_t bw) { return std::max<int64_t>(bw, 1) + 1; }
int64_t fl_band_stride(int64_t n, int64_t bw) { return ((fl_band_ldb(bw) * n + 31) / 32) * 32; }

hipError_t fl_band_factor(hipStream_t s, const fl_op* op, int64_t nshift, const double* sigma_dev, double* band,
                          double* lrow, int64_t* neg_dev) {
    const int64_t n = op->n, bw = std::max<int64_t>(op->inert_bw, 1);
    const int64_t ldb = fl_band_ldb(bw), stride = fl_band_stride(n, bw);
    hipError_t e = hipMemsetAsync(band, 0, (size_t)(nshift * stride) * 8, s);
    if (e != hipSuccess) return e;
    if ((e = hipMemsetAsync(lrow, 0, (size_t)(nshift * stride) * 8, s)) != hipSuccess) return e;
    band_build_kernel<<<dim3((unsigned)FL_DIV_UP(n, 256), (unsigned)nshift), 256, 0, s>>>(
        n, op->rowptr, op->colidx, op->kval, op->mval, op->inert_pinv, sigma_dev, ldb, stride, band);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    ldl_kernel<true><<<(unsigned)nshift, INT, 0, s>>>(n, (int)bw, ldb, stride, band, lrow, neg_dev);
    return hipGetLastError();
}

extern "C" {

int fl_inertia_count(fl_op* op, int64_t nshift, const double* sigma, int64_t* counts, int64_t* bandwidth_out) {
    if (!op) return FL_EINVAL;
    fl_ctx* ctx = op->ctx;
    if (nshift < 0 || (nshift > 0 && (!sigma || !counts)))
        return fl_fail(ctx, FL_EINVAL, "fl_inertia_count: bad arguments");
    for (int64_t s = 0; s < nshift; ++s)
        if (!std::isfinite(sigma[s])) return fl_fail(ctx, FL_EINVAL, "fl_inertia_count: non-finite shift");
    if (!op->rowptr) return fl_fail(ctx, FL_EINVAL, "fl_inertia_count: operator without a sparse pattern");
    FL_HIP(ctx, hipSetDevice(ctx->device));
    int rc = prepare_ordering(op);
    if (rc) return rc;
    if (bandwidth_out) *bandwidth_out = op->inert_bw;
    if (op->inert_bw > IBWMAX)
        return fl_fail(ctx, FL_EINVAL, "fl_inertia_count: bandwidth " + std::to_string(op->inert_bw) +
                                           " after reordering exceeds " + std::to_string(IBWMAX));
    if (nshift == 0) return FL_OK;
    const int64_t n = op->n, bw = std::max<int64_t>(op->inert_bw, 1);
    const int64_t ldb = bw + 1;
    const int64_t stride = ((ldb * n + 31) / 32) * 32;
    // shifts in batches that keep the bands under ~4 GiB
    const int64_t per = std::max<int64_t>(1, std::min<int64_t>(nshift, (int64_t(4) << 30) / (stride * 8)));
    DevBuf bband, bsig, bcnt;
    FL_HIP(ctx, bband.alloc((size_t)(per * stride) * 8));
    FL_HIP(ctx, bsig.alloc((size_t)per * 8));
    FL_HIP(ctx, bcnt.alloc((size_t)per * 8));
    hipStream_t s = ctx->stream;
    for (int64_t s0 = 0; s0 < nshift; s0 += per) {
        const int64_t ns = std::min(per, nshift - s0);
        FL_HIP(ctx, hipMemsetAsync(bband.p, 0, (size_t)(ns * stride) * 8, s));
        FL_HIP(ctx, hipMemcpyAsync(bsig.p, sigma + s0, ns * 8, hipMemcpyHostToDevice, s));
        band_build_kernel<<<dim3((unsigned)FL_DIV_UP(n, 256), (unsigned)ns), 256, 0, s>>>(
            n, op->rowptr, op->colidx, op->kval, op->mval, op->inert_pinv, bsig.as<double>(), ldb, stride,
            bband.as<double>());
        FL_HIP(ctx, hipGetLastError());
        ldl_kernel<false><<<(unsigned)ns, INT, 0, s>>>(n, (int)bw, ldb, stride, bband.as<double>(), nullptr,
                                                         bcnt.as<int64_t>());
        FL_HIP(ctx, hipGetLastError());
        FL_HIP(ctx, hipMemcpyAsync(counts + s0, bcnt.p, ns * 8, hipMemcpyDeviceToHost, s));
        FL_HIP(ctx, hipStreamSynchronize(s));
    }
    return FL_OK;
}

}  // extern "C"
