// Eigenpair refinement for the pencil (K, M) after Ogita and Aishima
// (iterative refinement for symmetric eigenvalue decomposition, JJIAM 2018),
// written in the M inner product that makes the eigenvectors orthonormal
// (Section "Post-processing").  With X the current approximate eigenvectors:
//   R = I - X^T M X,  S = X^T K X                (FP64; K X and M X from the
//                                                  sparse Galerkin matrices)
//   lambda_i = s_ii / (1 - r_ii)
//   E_ii = r_ii / 2
//   E_ij = (s_ij + lambda_j r_ij) / (lambda_j - lambda_i)   first-order rotation
//   E_ij = r_ij / 2  (no rotation) for pairs with
//        |lambda_i - lambda_j| <= delta = max(1e3 eps, sqrt(n) eps / tau) max|lambda|
//        (the rounding of s_ij, about sqrt(n) eps max|lambda|, would otherwise
//        rotate them by more than tau = 2e-6), and for near pairs
//        (gap < 1e-5 max|lambda|) whose first-order rotation exceeds tau.
//        Leaving such a pair mixed moves residuals, eigenvalues and solutions
//        by at most gap * |mixing|, below the FP64 targets.
//   X <- X + X E                                 (X kept in FP64; the
//        correction product runs on the FP32 matrix cores once
//        max|E| u_32 <= 5e-13, on the FP64 cores before)
// E_ij + E_ji = r_ij, so orthonormality is restored to second order; the
// off-diagonal error of X is roughly squared by each step.  The published
// cluster threshold 2(||S - diag(lambda)||_2 + max|lambda| ||R||_2) is not
// used: at large n it would treat most of the upper spectrum as one cluster.
// After the last step each column is scaled to unit M-norm and the
// eigenvalues are the Rayleigh quotients of the columns.
//
// Partial steps (partial > 0): every step after the first works on the
// lowest `partial` columns only, X_L <- X_L + X_L E_LL with R, S restricted
// to those columns, at O(n partial^2) instead of O(n^3).  This removes the
// second-order coupling error among the low modes (which dominates the
// fractional solutions) but not that of near-degenerate pairs higher in the
// spectrum, so the library's eigensolve uses full steps (partial = 0).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "internal.h"

namespace {

// lam_i = S_ii / R0_ii (R0 = X^T M X); max |I - R0| over the lower triangle,
// per block then reduced on the host
__global__ __launch_bounds__(256) void diag_kernel(int64_t n, const double* __restrict__ S, const double* __restrict__ R0,
                                                   int64_t ld, double* lam) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) lam[i] = S[i + i * ld] / R0[i + i * ld];
}

__global__ __launch_bounds__(256) void maxabs_offid_kernel(int64_t n, const double* __restrict__ R0, int64_t ld,
                                                           double* blockmax) {
    __shared__ double red[256];
    double m = 0.0;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)  // lower triangle (R0 is symmetric and stored there)
        for (int64_t j = blockIdx.y; j <= i; j += gridDim.y) m = fmax(m, fabs((i == j ? 1.0 : 0.0) - R0[i + j * ld]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) blockmax[blockIdx.x + (int64_t)blockIdx.y * gridDim.x] = red[0];
}

// E of the refinement step, one 32 x 32 tile of (i, j) per workgroup.  S and
// R = X^T M X hold only their lower triangles (the upper one is not
// formed), so every pair reads the same s_ij and r_ij from both sides: that
// keeps E_ij + E_ji = r_ij, the identity that preserves orthonormality (the
// GEMM would round S_ij and S_ji differently, and that difference divided by
// a small gap would break it).  A pair (i, j) is only re-orthonormalised
// (e = r/2, no rotation) when its gap is below delta, or when the gap is
// below gnear and the first-order rotation |e_ij| or |e_ji| exceeds tau
// (there the first-order formula is dominated by its second-order error).
// Pairs declined by the tau test are counted in nclus.
constexpr int ET = 32;
__global__ __launch_bounds__(256) void ebuild_kernel(int64_t n, const double* __restrict__ S,
                                                     const double* __restrict__ R0, int64_t ld,
                                                     const double* __restrict__ lam, double delta, double gnear,
                                                     double tau, double* E, int64_t lde, unsigned long long* nclus) {
    __shared__ double st[ET][ET + 1], rt[ET][ET + 1];  // transposed tiles S(J, I), R0(J, I)
    const int64_t i0 = (int64_t)blockIdx.x * ET, j0 = (int64_t)blockIdx.y * ET;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    // st[a][b] = S(j0 + a, i0 + b): coalesced along a
    for (int bb = ty; bb < ET; bb += 8) {
        const int64_t r = j0 + tx, c = i0 + bb;
        const bool ok = r < n && c < n;
        st[tx][bb] = ok ? S[r + c * ld] : 0.0;
        rt[tx][bb] = ok ? R0[r + c * ld] : 0.0;
    }
    __syncthreads();
    unsigned cnt = 0;
    const int64_t i = i0 + tx;
    if (i < n) {
        const double li = lam[i];
        for (int bb = ty; bb < ET; bb += 8) {
            const int64_t j = j0 + bb;
            if (j >= n) break;
            // lower triangle only: S_ij = S(max(i,j), min(i,j)), exactly symmetric
            const double sij = (i >= j) ? S[i + j * ld] : st[bb][tx];
            const double r = (i == j ? 1.0 : 0.0) - ((i >= j) ? R0[i + j * ld] : rt[bb][tx]);
            double e;
            if (i == j) {
                e = 0.5 * r;
            } else {
                const double lj = lam[j];
                const double g = lj - li;
                if (!(fabs(g) > delta)) {
                    e = 0.5 * r;
                } else {
                    const double eij = (sij + lj * r) / g;
                    const double eji = (sij + li * r) / (-g);
                    const bool clus = fabs(g) < gnear && (fabs(eij) > tau || fabs(eji) > tau);
                    e = clus ? 0.5 * r : eij;
                    if (clus && i < j) ++cnt;
                }
            }
            E[i + j * lde] = e;
        }
    }
    if (cnt) atomicAdd(nclus, (unsigned long long)cnt);
}

// theta_j = (x_j^T K x_j) / (x_j^T M x_j) from K X and M X, and x_j scaled to
// unit M-norm (one workgroup per column).  The scaling removes the diagonal
// of the second-order orthonormality error left by a step, sum_k e_kj^2,
// which grows with n (the off-diagonal terms are sums of mixed signs).
__global__ __launch_bounds__(256) void rq_kernel(int64_t n, double* __restrict__ X, int64_t ldx,
                                                 const double* __restrict__ KX, const double* __restrict__ MX,
                                                 int64_t ld, double* theta) {
    __shared__ double rk[256], rm[256];
    const int64_t j = blockIdx.x;
    double sk = 0.0, sm = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double x = X[i + j * ldx];
        sk += x * KX[i + j * ld];
        sm += x * MX[i + j * ld];
    }
    rk[threadIdx.x] = sk;
    rm[threadIdx.x] = sm;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            rk[threadIdx.x] += rk[threadIdx.x + w];
            rm[threadIdx.x] += rm[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) theta[j] = rk[0] / rm[0];
    const double sc = 1.0 / sqrt(rm[0]);
    for (int64_t i = threadIdx.x; i < n; i += 256) X[i + j * ldx] *= sc;
}

__global__ __launch_bounds__(256) void maxabs_kernel(int64_t m, int64_t n, const double* __restrict__ A, int64_t ld,
                                                     double* blockmax) {
    __shared__ double red[256];
    double mx = 0.0;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m)
        for (int64_t j = blockIdx.y; j < n; j += gridDim.y) mx = fmax(mx, fabs(A[i + j * ld]));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) blockmax[blockIdx.x + (int64_t)blockIdx.y * gridDim.x] = red[0];
}

__global__ void add_f_kernel(int64_t m, int64_t n, const float* __restrict__ D, int64_t ldd, double* X, int64_t ldx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        if (i < m) X[i + j * ldx] += (double)D[i + j * ldd];
}

// ranks of lam (ties by index), then permutation of columns
__global__ __launch_bounds__(256) void rank_kernel(int64_t n, const double* __restrict__ v, int64_t* rank) {
    __shared__ double tile[1024];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double vi = (i < n) ? v[i] : 0.0;
    int64_t r = 0;
    for (int64_t base = 0; base < n; base += 1024) {
        __syncthreads();
        for (int q = threadIdx.x; q < 1024; q += blockDim.x) tile[q] = (base + q < n) ? v[base + q] : 0.0;
        __syncthreads();
        int64_t lim = (n - base) < 1024 ? (n - base) : 1024;
        if (i < n)
            for (int64_t q = 0; q < lim; ++q) {
                double w = tile[q];
                r += (w < vi || (w == vi && base + q < i)) ? 1 : 0;
            }
    }
    if (i < n) rank[i] = r;
}

__global__ void permute_kernel(int64_t n, const int64_t* __restrict__ rank, const double* __restrict__ lin,
                               const double* __restrict__ Xin, int64_t ldin, double* lout, double* Xout, int64_t ldout) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t c = blockIdx.y; c < n; c += gridDim.y) {
        int64_t dst = rank[c];
        if (r < n) Xout[r + dst * ldout] = Xin[r + c * ldin];
        if (r == 0) lout[dst] = lin[c];
    }
}

inline dim3 g2(int64_t m, int64_t n) {
    return dim3((unsigned)FL_DIV_UP(m, 256), (unsigned)std::max<int64_t>(1, std::min<int64_t>(n, 65535)));
}

}  // namespace

// Refine (theta, X) in place.  X: n x n, ld ldx, approximately M-orthonormal
// eigenvectors of (K, M) given by op's CSR matrices.  max_iters steps at
// most; stops early when max |I - X^T M X| <= tol.  theta (n) receives the
// refined eigenvalues, ascending (columns of X permuted to match).
// Eigenvalues of the columns of X as Rayleigh quotients x^T K x / x^T M x
// with the sparse K and M, columns scaled to unit M-norm, then sorted
// ascending (O(n^2) work: two sparse products and column reductions).
int fl_rayleigh_device(fl_ctx* ctx, fl_op* op, double* theta, double* X, int64_t ldx) {
    hipStream_t s = ctx->stream;
    const int64_t n = op->n;
    DevBuf bKX, bMX, bv;
    FL_HIP(ctx, bKX.alloc(sizeof(double) * n * n));
    FL_HIP(ctx, bMX.alloc(sizeof(double) * n * n));
    FL_HIP(ctx, bv.alloc(sizeof(double) * n + sizeof(int64_t) * n));
    double* KX = bKX.as<double>();
    double* MX = bMX.as<double>();
    double* lam2 = bv.as<double>();
    int64_t* rank = reinterpret_cast<int64_t*>(lam2 + n);
    FL_HIP(ctx, fl_spmm_csr(s, n, op->rowptr, op->colidx, op->kval, n, X, ldx, KX, n));
    FL_HIP(ctx, fl_spmm_csr(s, n, op->rowptr, op->colidx, op->mval, n, X, ldx, MX, n));
    rq_kernel<<<(unsigned)n, 256, 0, s>>>(n, X, ldx, KX, MX, n, theta);
    FL_HIP(ctx, hipGetLastError());
    rank_kernel<<<(unsigned)FL_DIV_UP(n, 256), 256, 0, s>>>(n, theta, rank);
    FL_HIP(ctx, hipGetLastError());
    permute_kernel<<<g2(n, n), 256, 0, s>>>(n, rank, theta, X, ldx, lam2, KX, n);
    FL_HIP(ctx, hipGetLastError());
    FL_HIP(ctx, hipMemcpy2DAsync(X, ldx * 8, KX, n * 8, n * 8, n, hipMemcpyDeviceToDevice, s));
    FL_HIP(ctx, hipMemcpyAsync(theta, lam2, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    FL_HIP(ctx, hipStreamSynchronize(s));
    return FL_OK;
}

int fl_refine_device(fl_ctx* ctx, fl_op* op, double* theta, double* X, int64_t ldx, int max_iters, double tol,
                     fl_eig_info* info, int64_t partial) {
    hipStream_t s = ctx->stream;
    const int64_t n = op->n;
    const int64_t ld = n;
    DevBuf bKX, bMX, bS, bR, bE, bXf, bXEf, bv;
    FL_HIP(ctx, bKX.alloc(sizeof(double) * n * n));
    FL_HIP(ctx, bMX.alloc(sizeof(double) * n * n));
    FL_HIP(ctx, bS.alloc(sizeof(double) * n * n));
    FL_HIP(ctx, bR.alloc(sizeof(double) * n * n));
    FL_HIP(ctx, bE.alloc(sizeof(double) * n * n));
    FL_HIP(ctx, bXf.alloc(sizeof(float) * n * n));
    FL_HIP(ctx, bXEf.alloc(sizeof(float) * n * n));
    const int64_t nbm = FL_DIV_UP(n, 256) * std::min<int64_t>(n, 1024);
    FL_HIP(ctx, bv.alloc(sizeof(double) * (2 * n + nbm) + sizeof(int64_t) * n + 64));
    double* KX = bKX.as<double>();
    double* MX = bMX.as<double>();
    double* S = bS.as<double>();
    double* R0 = bR.as<double>();
    double* E = bE.as<double>();
    float* Xf = bXf.as<float>();
    float* XEf = bXEf.as<float>();
    double* lam = bv.as<double>();
    double* lam2 = lam + n;
    double* bmax = lam2 + n;
    int64_t* rank = (int64_t*)(bmax + nbm);
    unsigned long long* nclus = (unsigned long long*)(rank + n);
    const bool verbose = getenv("FRACLAP_VERBOSE") != nullptr;
    const dim3 gm((unsigned)FL_DIV_UP(n, 256), (unsigned)std::min<int64_t>(n, 1024));
    std::vector<double> hb((size_t)gm.x * gm.y);
    // max over the per-block maxima of a launch on grid g
    auto reduce_max = [&](const dim3& g, double* out) -> int {
        const size_t cnt = (size_t)g.x * g.y;
        FL_HIP(ctx, hipMemcpyAsync(hb.data(), bmax, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));
        FL_HIP(ctx, hipStreamSynchronize(s));
        double m = 0.0;
        for (size_t q = 0; q < cnt; ++q) m = std::max(m, hb[q]);
        *out = m;
        return FL_OK;
    };
    int iters = 0;
    double resid = -1.0;
    bool updated = false;  // X changed since theta was last computed
    for (int it = 0; it < max_iters; ++it) {
        // the first step works on every column; later steps, if partial > 0,
        // only on the lowest `partial` columns (see the header)
        const int64_t kc = (it == 0 || partial <= 0) ? n : std::min<int64_t>(n, partial);
        const dim3 gk((unsigned)FL_DIV_UP(kc, 256), (unsigned)std::min<int64_t>(kc, 1024));
        FL_HIP(ctx, fl_spmm_csr(s, n, op->rowptr, op->colidx, op->kval, kc, X, ldx, KX, ld));
        FL_HIP(ctx, fl_spmm_csr(s, n, op->rowptr, op->colidx, op->mval, kc, X, ldx, MX, ld));
        // S and X^T M X are symmetric: only their lower triangles are formed
        FL_HIP(ctx, fl_dgemm(s, 1, 0, kc, kc, n, 1.0, X, ldx, KX, ld, 0.0, S, ld, 1));
        FL_HIP(ctx, fl_dgemm(s, 1, 0, kc, kc, n, 1.0, X, ldx, MX, ld, 0.0, R0, ld, 1));
        diag_kernel<<<(unsigned)FL_DIV_UP(kc, 256), 256, 0, s>>>(kc, S, R0, ld, lam);
        FL_HIP(ctx, hipGetLastError());
        FL_HIP(ctx, hipMemcpyAsync(theta, lam, sizeof(double) * kc, hipMemcpyDeviceToDevice, s));
        updated = false;
        maxabs_offid_kernel<<<gk, 256, 0, s>>>(kc, R0, ld, bmax);
        FL_HIP(ctx, hipGetLastError());
        double mr = 0.0, lmax = 0.0;
        if (int rc = reduce_max(gk, &mr)) return rc;
        maxabs_kernel<<<gk, 256, 0, s>>>(kc, 1, lam, kc, bmax);
        FL_HIP(ctx, hipGetLastError());
        if (int rc = reduce_max(gk, &lmax)) return rc;
        if (kc == n) resid = mr;
        if (mr <= tol) break;
        // delta: below this gap the rounding of S (about sqrt(n) eps max|lambda|)
        // divided by the gap would rotate by more than tau, so such pairs count
        // as degenerate; gnear, tau: a near pair whose rotation exceeds tau
        // is dominated by the second-order term and is left unrotated
        const double tau = 2e-6;
        const double delta = std::max(1e3 * 2.220446049250313e-16,
                                      std::sqrt((double)n) * 2.220446049250313e-16 / tau) * lmax;
        const double gnear = 1e-5 * lmax;
        FL_HIP(ctx, hipMemsetAsync(nclus, 0, sizeof(unsigned long long), s));
        const dim3 ge((unsigned)FL_DIV_UP(kc, ET), (unsigned)FL_DIV_UP(kc, ET));
        ebuild_kernel<<<ge, 256, 0, s>>>(kc, S, R0, ld, lam, delta, gnear, tau, E, n, nclus);
        FL_HIP(ctx, hipGetLastError());
        maxabs_kernel<<<gk, 256, 0, s>>>(kc, kc, E, n, bmax);
        FL_HIP(ctx, hipGetLastError());
        double emax = 0.0;
        if (int rc = reduce_max(gk, &emax)) return rc;
        if (verbose) {
            unsigned long long nc = 0;
            FL_HIP(ctx, hipMemcpy(&nc, nclus, sizeof(nc), hipMemcpyDeviceToHost));
            fprintf(stderr,
                    "[fraclap] refine step %d on %lld columns: max|I - X^T M X| %.3e  max|E| %.3e  tau-clustered pairs %llu\n",
                    it, (long long)kc, mr, emax, nc);
        }
        if (emax * 6.0e-8 <= 5e-13) {
            // X += X E on the FP32 matrix cores: the product's rounding,
            // about u_32 max|E| relative to X, stays below the FP64 targets
            // for orthonormality and residual (and enters the eigenvalues
            // only squared)
            float* Ef = reinterpret_cast<float*>(MX);  // M X is consumed: reuse its space
            FL_HIP(ctx, fl_d2s(s, n, kc, X, ldx, Xf, n));
            FL_HIP(ctx, fl_d2s(s, kc, kc, E, n, Ef, kc));
            FL_HIP(ctx, fl_sgemm(s, 0, 0, n, kc, kc, 1.0f, Xf, n, Ef, kc, 0.0f, XEf, n));
            add_f_kernel<<<g2(n, kc), 256, 0, s>>>(n, kc, XEf, n, X, ldx);
            FL_HIP(ctx, hipGetLastError());
        } else {
            // X += X E in FP64: X_old copied into the (consumed) M X buffer
            FL_HIP(ctx, hipMemcpy2DAsync(MX, ld * 8, X, ldx * 8, n * 8, kc, hipMemcpyDeviceToDevice, s));
            FL_HIP(ctx, fl_dgemm(s, 0, 0, n, kc, kc, 1.0, MX, ld, E, n, 1.0, X, ldx));
        }
        updated = true;
        ++iters;
    }
    if (updated) {
        // eigenvalues of the final X: column Rayleigh quotients, and unit
        // M-norms (O(n^2) work)
        FL_HIP(ctx, fl_spmm_csr(s, n, op->rowptr, op->colidx, op->kval, n, X, ldx, KX, ld));
        FL_HIP(ctx, fl_spmm_csr(s, n, op->rowptr, op->colidx, op->mval, n, X, ldx, MX, ld));
        rq_kernel<<<(unsigned)n, 256, 0, s>>>(n, X, ldx, KX, MX, ld, theta);
        FL_HIP(ctx, hipGetLastError());
    }
    // ascending order (refinement may swap nearly equal neighbours)
    rank_kernel<<<(unsigned)FL_DIV_UP(n, 256), 256, 0, s>>>(n, theta, rank);
    FL_HIP(ctx, hipGetLastError());
    permute_kernel<<<g2(n, n), 256, 0, s>>>(n, rank, theta, X, ldx, lam2, KX, ld);
    FL_HIP(ctx, hipGetLastError());
    FL_HIP(ctx, hipMemcpy2DAsync(X, ldx * 8, KX, ld * 8, n * 8, n, hipMemcpyDeviceToDevice, s));
    FL_HIP(ctx, hipMemcpyAsync(theta, lam2, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    FL_HIP(ctx, hipStreamSynchronize(s));
    if (info) {
        info->refine_iters = iters;
        info->refine_resid = resid;
    }
    return FL_OK;
}
