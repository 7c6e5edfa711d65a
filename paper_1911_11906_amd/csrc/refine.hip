// Eigenpair refinement for the pencil (K, M) after Ogita and Aishima
// (iterative refinement for symmetric eigenvalue decomposition, JJIAM 2018),
// written in the M inner product that makes the eigenvectors orthonormal
// (Section "Post-processing").  With X the current approximate eigenvectors:
//   R = I - X^T M X,  S = X^T K X                (FP64; K X and M X from the
//                                                  sparse Galerkin matrices)
//   lambda_i = s_ii / (1 - r_ii)
//   E_ii = r_ii / 2
//   E_ij = (s_ij + lambda_j r_ij) / (lambda_j - lambda_i)  if |lambda_i - lambda_j| > delta
//        = r_ij / 2                                        otherwise (cluster)
//   delta = 1e3 eps max|lambda|: pairs closer than the rounding level of the
//           lambda are (exactly) degenerate and are only re-orthonormalised.
//           The published sufficient threshold 2(||S - diag(lambda)||_2 +
//           max|lambda| ||R||_2) is far larger for FP32 starting vectors at
//           large n (it would freeze most of the upper spectrum); the update
//           converges whenever the mixing angle of a pair is small, which the
//           FP32 reduction delivers, so the rounding level is used.
//   X <- X + X E                                 (X kept in FP64; the
//        correction product runs on the FP32 matrix cores once
//        max|E| u_32 is below the FP64 target, on the FP64 cores before)
// Each step roughly squares the error of X.  The refined eigenvalues are the
// lambda of the last step (Rayleigh-quotient accurate).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "internal.h"

namespace {

// lam_i = S_ii / R0_ii (R0 = X^T M X); mx = max |I - R0|, per block then reduced
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
    if (i < n)
        for (int64_t j = blockIdx.y; j < n; j += gridDim.y) m = fmax(m, fabs((i == j ? 1.0 : 0.0) - R0[i + j * ld]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) blockmax[blockIdx.x + (int64_t)blockIdx.y * gridDim.x] = red[0];
}

// y = (A - diag(d)) x  or  y = x - A x (mode 1), after y = A x by GEMM
__global__ void shift_kernel(int64_t n, int mode, const double* __restrict__ x, const double* __restrict__ d,
                             double* y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = (mode == 0) ? y[i] - d[i] * x[i] : x[i] - y[i];
}

__global__ __launch_bounds__(256) void norm2_kernel(int64_t n, const double* __restrict__ x, double* out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i] * x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sqrt(red[0]);
}

__global__ void scale_kernel(int64_t n, const double* __restrict__ nrm, const double* __restrict__ y, double* x) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = (nrm[0] > 0.0) ? y[i] / nrm[0] : 0.0;
}

// E of the refinement step.  A pair (i, j) is clustered when the lambdas
// agree to the rounding level delta, or when the first-order rotation
// |e_ij| or |e_ji| exceeds tau (the pair is not yet separated well enough for
// a first-order correction); clustered pairs are only re-orthonormalised
// here (e = r/2) and appended to `pairs` (i < j) for the Rayleigh-Ritz step.
__global__ void ebuild_kernel(int64_t n, const double* __restrict__ S, const double* __restrict__ R0, int64_t ld,
                              const double* __restrict__ lam, double delta, double tau, double* E, int64_t lde,
                              int64_t* pairs, unsigned long long* npairs, int64_t cap) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double li = lam[i];
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
        double r = (i == j ? 1.0 : 0.0) - R0[i + j * ld];
        double e;
        if (i == j) {
            e = 0.5 * r;
        } else {
            const double lj = lam[j];
            const double g = lj - li;
            const double sij = S[i + j * ld];
            const double eij = (sij + lj * r) / g;
            const double eji = (sij + li * r) / (-g);
            const bool clus = !(fabs(g) > delta) || fabs(eij) > tau || fabs(eji) > tau;
            e = clus ? 0.5 * r : eij;
            if (clus && i < j) {
                unsigned long long k = atomicAdd(npairs, 1ull);
                if ((int64_t)k < cap) {
                    pairs[2 * k] = i;
                    pairs[2 * k + 1] = j;
                }
            }
        }
        E[i + j * lde] = e;
    }
}

// Rayleigh-Ritz on one cluster (one workgroup of 64 threads): with
// P = X_c^T K X_c and Q = X_c^T M X_c (c x c), Q = L L^T, solve
// L^-1 P L^-T = W diag(mu) W^T by cyclic Jacobi, Y = L^-T W (ascending mu).
constexpr int RRMAX = 80;
__global__ __launch_bounds__(64) void rr_small_kernel(const int64_t* __restrict__ coff, const double* __restrict__ PQ,
                                                      double* Y, double* mu) {
    __shared__ double A[RRMAX * RRMAX], L[RRMAX * RRMAX], W[RRMAX * RRMAX];
    __shared__ double cs[2];
    __shared__ int more;
    const int t = threadIdx.x;
    const int64_t o = coff[blockIdx.x];
    const int c = (int)(coff[blockIdx.x + 1] - o);
    const double* P = PQ + 2 * o * RRMAX;            // c x c, ld c  (packed by cluster)
    const double* Q = P + (int64_t)c * c;
    for (int e = t; e < c * c; e += 64) {
        A[e] = P[e];
        L[e] = Q[e];
    }
    __syncthreads();
    // Cholesky of Q (lower, in L), column by column
    for (int j = 0; j < c; ++j) {
        if (t == 0) {
            double d = L[j + j * c];
            for (int k = 0; k < j; ++k) d -= L[j + k * c] * L[j + k * c];
            L[j + j * c] = sqrt(d > 0.0 ? d : 1e-300);
        }
        __syncthreads();
        for (int i = j + 1 + t; i < c; i += 64) {
            double v = L[i + j * c];
            for (int k = 0; k < j; ++k) v -= L[i + k * c] * L[j + k * c];
            L[i + j * c] = v / L[j + j * c];
        }
        __syncthreads();
    }
    // A := L^-1 A L^-T : columns of A by forward substitution, then rows
    for (int col = t; col < c; col += 64)
        for (int i = 0; i < c; ++i) {
            double v = A[i + col * c];
            for (int k = 0; k < i; ++k) v -= L[i + k * c] * A[k + col * c];
            A[i + col * c] = v / L[i + i * c];
        }
    __syncthreads();
    for (int row = t; row < c; row += 64)
        for (int i = 0; i < c; ++i) {
            double v = A[row + i * c];
            for (int k = 0; k < i; ++k) v -= L[i + k * c] * A[row + k * c];
            A[row + i * c] = v / L[i + i * c];
        }
    __syncthreads();
    for (int e = t; e < c * c; e += 64) W[e] = ((e % c) == (e / c)) ? 1.0 : 0.0;
    __syncthreads();
    // cyclic Jacobi (row-by-row ordering), rotations applied by all threads
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (t == 0) more = 0;
        __syncthreads();
        for (int p = 0; p < c - 1; ++p)
            for (int q = p + 1; q < c; ++q) {
                if (t == 0) {
                    double apq = A[p + q * c], app = A[p + p * c], aqq = A[q + q * c];
                    double cc = 1.0, ss = 0.0;
                    if (fabs(apq) > 2.220446049250313e-16 * sqrt(fabs(app * aqq)) && apq != 0.0) {
                        double th = (aqq - app) / (2.0 * apq);
                        double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
                        cc = 1.0 / sqrt(1.0 + tt * tt);
                        ss = tt * cc;
                        more = 1;
                    }
                    cs[0] = cc;
                    cs[1] = ss;
                }
                __syncthreads();
                const double cc = cs[0], ss = cs[1];
                if (ss != 0.0) {
                    for (int k = t; k < c; k += 64) {  // columns p, q
                        double x = A[k + p * c], y = A[k + q * c];
                        A[k + p * c] = cc * x - ss * y;
                        A[k + q * c] = ss * x + cc * y;
                        double u = W[k + p * c], w = W[k + q * c];
                        W[k + p * c] = cc * u - ss * w;
                        W[k + q * c] = ss * u + cc * w;
                    }
                    __syncthreads();
                    for (int k = t; k < c; k += 64) {  // rows p, q
                        double x = A[p + k * c], y = A[q + k * c];
                        A[p + k * c] = cc * x - ss * y;
                        A[q + k * c] = ss * x + cc * y;
                    }
                }
                __syncthreads();
            }
        if (!more) break;
    }
    // Y = L^-T W, columns sorted by ascending mu (selection by rank)
    for (int col = t; col < c; col += 64)
        for (int i = c - 1; i >= 0; --i) {
            double v = W[i + col * c];
            for (int k = i + 1; k < c; ++k) v -= L[k + i * c] * W[k + col * c];
            W[i + col * c] = v / L[i + i * c];
        }
    __syncthreads();
    for (int col = t; col < c; col += 64) {
        double m = A[col + col * c];
        int rnk = 0;
        for (int k = 0; k < c; ++k) {
            double mk = A[k + k * c];
            rnk += (mk < m || (mk == m && k < col)) ? 1 : 0;
        }
        mu[o + rnk] = m;
        for (int i = 0; i < c; ++i) Y[o * RRMAX + i + (int64_t)rnk * c] = W[i + col * c];
    }
}

__global__ void gather_cols_kernel(int64_t n, int64_t m, const int64_t* __restrict__ idx, const double* __restrict__ X,
                                   int64_t ldx, double* Xc) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t c = blockIdx.y; c < m; c += gridDim.y)
        if (r < n) Xc[r + c * n] = X[r + idx[c] * ldx];
}

__global__ void scatter_cols_kernel(int64_t n, int64_t m, const int64_t* __restrict__ idx, const double* __restrict__ Xc,
                                    double* X, int64_t ldx, const double* __restrict__ mu, double* theta) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t c = blockIdx.y; c < m; c += gridDim.y) {
        if (r < n) X[r + idx[c] * ldx] = Xc[r + c * n];
        if (r == 0) theta[idx[c]] = mu[c];
    }
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

// 2-norm estimate of (A - diag(d)) (mode 0) or (I - A) (mode 1), A symmetric
// n x n (ld), by `iters` power iterations from a fixed start vector.
[[maybe_unused]] static int norm2_est(fl_ctx* ctx, int64_t n, const double* A, int64_t ld, const double* d, int mode, int iters,
                     double* xv, double* yv, double* nrm, double* out) {
    hipStream_t s = ctx->stream;
    std::vector<double> x0(n);
    for (int64_t i = 0; i < n; ++i) x0[i] = 1.0 + 0.37 * std::sin(0.731 * (double)i + 0.2);
    double s2 = 0.0;
    for (double v : x0) s2 += v * v;
    for (double& v : x0) v /= std::sqrt(s2);
    FL_HIP(ctx, hipMemcpyAsync(xv, x0.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
    double est = 0.0;
    for (int it = 0; it < iters; ++it) {
        FL_HIP(ctx, fl_dgemm(s, 0, 0, n, 1, n, 1.0, A, ld, xv, n, 0.0, yv, n));
        shift_kernel<<<(unsigned)FL_DIV_UP(n, 256), 256, 0, s>>>(n, mode, xv, d, yv);
        FL_HIP(ctx, hipGetLastError());
        norm2_kernel<<<1, 256, 0, s>>>(n, yv, nrm);
        FL_HIP(ctx, hipGetLastError());
        scale_kernel<<<(unsigned)FL_DIV_UP(n, 256), 256, 0, s>>>(n, nrm, yv, xv);
        FL_HIP(ctx, hipGetLastError());
    }
    FL_HIP(ctx, hipMemcpyAsync(&est, nrm, sizeof(double), hipMemcpyDeviceToHost, s));
    FL_HIP(ctx, hipStreamSynchronize(s));
    *out = est;
    return FL_OK;
}

// Refine (theta, X) in place.  X: n x n, ld ldx, approximately M-orthonormal
// eigenvectors of (K, M) given by op's CSR matrices.  max_iters steps at
// most; stops early when max |I - X^T M X| <= tol.  theta (n) receives the
// refined eigenvalues, ascending (columns of X permuted to match).
int fl_refine_device(fl_ctx* ctx, fl_op* op, double* theta, double* X, int64_t ldx, int max_iters, double tol,
                     fl_eig_info* info) {
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
    FL_HIP(ctx, bv.alloc(sizeof(double) * (4 * n + 8 + nbm) + sizeof(int64_t) * n + 64));
    double* KX = bKX.as<double>();
    double* MX = bMX.as<double>();
    double* S = bS.as<double>();
    double* R0 = bR.as<double>();
    double* E = bE.as<double>();
    float* Xf = bXf.as<float>();
    float* Ef = bXf.as<float>();  // reassigned below (Xf and Ef need separate space)
    float* XEf = bXEf.as<float>();
    double* lam = bv.as<double>();
    double* xv = lam + n;
    double* yv = xv + n;
    double* lam2 = yv + n;
    double* nrm = lam2 + n;
    double* bmax = nrm + 8;
    int64_t* rank = (int64_t*)(bmax + nbm);
    unsigned long long* npairs = (unsigned long long*)(rank + n);
    int iters = 0;
    double resid = -1.0;
    for (int it = 0; it < max_iters; ++it) {
        FL_HIP(ctx, fl_spmm_csr(s, n, op->rowptr, op->colidx, op->kval, n, X, ldx, KX, ld));
        FL_HIP(ctx, fl_spmm_csr(s, n, op->rowptr, op->colidx, op->mval, n, X, ldx, MX, ld));
        FL_HIP(ctx, fl_dgemm(s, 1, 0, n, n, n, 1.0, X, ldx, KX, ld, 0.0, S, ld));
        FL_HIP(ctx, fl_dgemm(s, 1, 0, n, n, n, 1.0, X, ldx, MX, ld, 0.0, R0, ld));
        diag_kernel<<<(unsigned)FL_DIV_UP(n, 256), 256, 0, s>>>(n, S, R0, ld, lam);
        FL_HIP(ctx, hipGetLastError());
        // max |I - X^T M X|
        dim3 gm((unsigned)FL_DIV_UP(n, 256), (unsigned)std::min<int64_t>(n, 1024));
        maxabs_offid_kernel<<<gm, 256, 0, s>>>(n, R0, ld, bmax);
        FL_HIP(ctx, hipGetLastError());
        std::vector<double> hb((size_t)gm.x * gm.y);
        FL_HIP(ctx, hipMemcpyAsync(hb.data(), bmax, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, s));
        std::vector<double> hl(n);
        FL_HIP(ctx, hipMemcpyAsync(hl.data(), lam, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        FL_HIP(ctx, hipStreamSynchronize(s));
        double mr = 0.0, lmax = 0.0;
        for (double v : hb) mr = std::max(mr, v);
        for (double v : hl) lmax = std::max(lmax, std::fabs(v));
        resid = mr;
        FL_HIP(ctx, hipMemcpyAsync(theta, lam, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        if (mr <= tol) break;
        const double delta = 1e3 * 2.220446049250313e-16 * lmax;
        ebuild_kernel<<<g2(n, n), 256, 0, s>>>(n, S, R0, ld, lam, delta, INFINITY, E, n, nullptr, npairs, 0);
        FL_HIP(ctx, hipGetLastError());
        maxabs_kernel<<<gm, 256, 0, s>>>(n, n, E, n, bmax);
        FL_HIP(ctx, hipGetLastError());
        FL_HIP(ctx, hipMemcpyAsync(hb.data(), bmax, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, s));
        FL_HIP(ctx, hipStreamSynchronize(s));
        double emax = 0.0;
        for (double v : hb) emax = std::max(emax, v);
        if (getenv("FRACLAP_VERBOSE"))
            fprintf(stderr, "[fraclap] refine step %d: max|I - X^T M X| %.3e  max|E| %.3e  delta %.3e\n", it, mr, emax,
                    delta);
        if (emax * 6.0e-8 <= 1e-14) {
            // X += X E on the FP32 matrix cores (E and the FP32 rounding of X
            // are both small enough for an FP64-accurate correction)
            Ef = reinterpret_cast<float*>(MX);  // M X is consumed: reuse its space
            FL_HIP(ctx, fl_d2s(s, n, n, X, ldx, Xf, n));
            FL_HIP(ctx, fl_d2s(s, n, n, E, n, Ef, n));
            FL_HIP(ctx, fl_sgemm(s, 0, 0, n, n, n, 1.0f, Xf, n, Ef, n, 0.0f, XEf, n));
            add_f_kernel<<<g2(n, n), 256, 0, s>>>(n, n, XEf, n, X, ldx);
            FL_HIP(ctx, hipGetLastError());
        } else {
            // X += X E in FP64: X_old copied into the (consumed) M X buffer
            FL_HIP(ctx, hipMemcpy2DAsync(MX, ld * 8, X, ldx * 8, n * 8, n, hipMemcpyDeviceToDevice, s));
            FL_HIP(ctx, fl_dgemm(s, 0, 0, n, n, n, 1.0, MX, ld, E, n, 1.0, X, ldx));
        }
        ++iters;
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
