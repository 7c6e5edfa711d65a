// Spectral application v = sum_k theta_k^(-alpha/2) (phi_k^T M f) phi_k
// (Section "Method", equations for g and v) and its adjoint.
//
//   G = M F            CSR SpMM (HBM bound)
//   C = V^T G          FP64 MFMA GEMM
//   W_ki = exp(-(alpha_i/2) ln theta_k)       (alpha = 0 gives exactly 1);
//        for the diffusion equation (Section "Method", equation
//        diffusion_solution) W_ki = exp(-mu_i t_i theta_k^(alpha_i/2))
//   U[:, j + i nf] = V (W[:, i] o C[:, j])    one FP64 MFMA GEMM whose
//        operand B is formed while it is staged into LDS, so the
//        na-times-larger scaled operand never exists in memory.
// Adjoint (paired pairs b): P = V^T GU, GF = M V (W o P), and the
// derivative with respect to each weight parameter
//   g_b = sum_k P_kb C_kb dW_kb/dparam_b.
#include "internal.h"
#include "gemm_tile.h"

namespace {
using namespace fl_tile;

// Y = A X for CSR A (n x n) and dense X (n x ncols).  A thread takes one row
// and SPC columns, so each stored entry is read once per SPC columns.
constexpr int SPC = 8;
__global__ void spmm_kernel(int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                            const double* __restrict__ val, int64_t ncols, const double* __restrict__ X, int64_t ldx,
                            double* __restrict__ Y, int64_t ldy) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t p0 = rowptr[i], p1 = rowptr[i + 1];
    for (int64_t c0 = (int64_t)blockIdx.y * SPC; c0 < ncols; c0 += (int64_t)gridDim.y * SPC) {
        const int nc = (int)((ncols - c0) < SPC ? (ncols - c0) : SPC);
        double s[SPC];
#pragma unroll
        for (int c = 0; c < SPC; ++c) s[c] = 0.0;
        for (int32_t p = p0; p < p1; ++p) {
            const double v = val[p];
            const double* x = X + colidx[p] + c0 * ldx;
#pragma unroll
            for (int c = 0; c < SPC; ++c)
                if (c < nc) s[c] += v * x[c * ldx];
        }
#pragma unroll
        for (int c = 0; c < SPC; ++c)
            if (c < nc) Y[i + (c0 + c) * ldy] = s[c];
    }
}

__global__ void log_kernel(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = log(x[i]);
}

// Spectral weights W[k, i] of one chunk of columns, parameters passed by value
// (nothing is copied from the host, so the sequence can be captured in a
// graph).  FL_SPEC_FRACTIONAL: W = theta^(-alpha/2) = exp(-(alpha/2) ln theta)
// (alpha = 0 gives exactly 1).  FL_SPEC_DIFFUSION: W = exp(-s theta^(alpha/2))
// with s = mu t (the solution of the diffusion equation at time t).
__global__ void weights_kernel(int64_t n, const double* __restrict__ logtheta, WeightArgs a,
                               double* __restrict__ W, int64_t ldw) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double lt = logtheta[k];
    for (int i = blockIdx.y; i < a.count; i += gridDim.y) {
        const double e = exp(0.5 * a.alpha[i] * lt);  // theta^(alpha/2)
        W[k + i * ldw] = a.kind == FL_SPEC_DIFFUSION ? exp(-a.s[i] * e) : exp(-0.5 * a.alpha[i] * lt);
    }
}

// op(B)[kk][col] = W[kk, i(col)] * C[kk, j(col)], col = j + i nf (paired: i = j = col)
struct BScaled {
    const double* W;
    int64_t ldw;
    const double* Cc;
    int64_t ldc;
    int64_t nf;
    int paired;
    struct H {
        const double* w;
        const double* c;
    };
    __device__ inline H col(int64_t col) const {
        int64_t i = paired ? col : col / nf;
        int64_t j = paired ? col : col - i * nf;
        return H{W + i * ldw, Cc + j * ldc};
    }
    __device__ inline double at(const H& h, int64_t kk) const { return h.w[kk] * h.c[kk]; }
    static constexpr bool KSCALE = false;
    __device__ inline const double* kcol(int64_t) const { return nullptr; }
    __device__ inline double kscale(const double*, int64_t) const { return 1.0; }
};

// Same operand when every column of a 128-wide tile has the same alpha
// (all pairs with nf a multiple of 128): the weight is one number per
// (tile, k-row), loaded once per k-step instead of once per element.
struct BScaledUniform {
    const double* W;
    int64_t ldw;
    const double* Cc;
    int64_t ldc;
    int64_t nf;
    struct H {
        const double* c;
    };
    __device__ inline H col(int64_t col) const {
        int64_t i = col / nf;
        return H{Cc + (col - i * nf) * ldc};
    }
    __device__ inline double at(const H& h, int64_t kk) const { return h.c[kk]; }
    static constexpr bool KSCALE = true;
    // the weight column of the tile's alpha (one index division per tile)
    __device__ inline const double* kcol(int64_t col0) const { return W + (col0 / nf) * ldw; }
    __device__ inline double kscale(const double* wc, int64_t kk) const { return wc[kk]; }
};

template <class BS, int KB>
__global__ __launch_bounds__(NT) FL_TWO_WAVES_PER_SIMD void scaled_gemm_kernel(int64_t n, int64_t ncol,
                                                                            const double* __restrict__ V,
                                                                            int64_t ldv, BS bs, double* __restrict__ U,
                                                                            int64_t ldu, int64_t group) {
    __shared__ double As[TileLds<KB, 1>::A];
    __shared__ double Bs[TileLds<KB, 1>::B];
    int64_t bi, bj;
    xcd_grouped_tile(bi, bj, group);
    tile_gemm<false, true, BS, KB, 1>(n, ncol, n, V, ldv, bs, 1.0, 0.0, U, ldu, bi, bj, As, Bs);
}

// Derivatives of the paired map with respect to the weight parameters, one
// block per column b of the chunk, fixed-order tree reduction
// (deterministic):  with q_k = P[k,b] C[k,b] W[k,b],
//   FL_SPEC_FRACTIONAL: ga[b] = sum_k q_k (-ln theta_k / 2)
//   FL_SPEC_DIFFUSION:  ga[b] = sum_k q_k (-s_b theta_k^(alpha_b/2) ln theta_k / 2),
//                       gs[b] = sum_k q_k (-theta_k^(alpha_b/2))
__global__ __launch_bounds__(256) void spec_grad_kernel(int64_t n, const double* __restrict__ P, int64_t ldp,
                                                        const double* __restrict__ C, int64_t ldc,
                                                        const double* __restrict__ W, int64_t ldw,
                                                        const double* __restrict__ logtheta, WeightArgs a,
                                                        double* ga, double* gs) {
    __shared__ double red[2][256];
    const int b = blockIdx.x;
    const bool dif = a.kind == FL_SPEC_DIFFUSION;
    double sa = 0.0, ss = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += 256) {
        const double lt = logtheta[k];
        const double q = P[k + b * ldp] * W[k + b * ldw] * C[k + b * ldc];
        if (dif) {
            const double e = exp(0.5 * a.alpha[b] * lt);
            sa += q * (-0.5 * a.s[b] * e * lt);
            ss += q * (-e);
        } else {
            sa += q * (-0.5 * lt);
        }
    }
    red[0][threadIdx.x] = sa;
    red[1][threadIdx.x] = ss;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ga[b] = red[0][0];
        if (gs) gs[b] = red[1][0];
    }
}

__global__ void finite_kernel(int64_t m, int64_t n, const double* __restrict__ A, int64_t lda, int* flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        if (!isfinite(A[i + j * lda])) {
            __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
}

}  // namespace

hipError_t fl_spmm_csr(hipStream_t s, int64_t n, const int32_t* rowptr, const int32_t* colidx, const double* val,
                       int64_t ncols, const double* X, int64_t ldx, double* Y, int64_t ldy) {
    if (n <= 0 || ncols <= 0) return hipSuccess;
    const int64_t cg = FL_DIV_UP(ncols, SPC);
    dim3 grid((unsigned)FL_DIV_UP(n, 256), (unsigned)(cg < 65535 ? cg : 65535));
    spmm_kernel<<<grid, 256, 0, s>>>(n, rowptr, colidx, val, ncols, X, ldx, Y, ldy);
    return hipGetLastError();
}

hipError_t fl_log_kernel(hipStream_t s, int64_t n, const double* x, double* y) {
    if (n <= 0) return hipSuccess;
    log_kernel<<<(unsigned)FL_DIV_UP(n, 256), 256, 0, s>>>(n, x, y);
    return hipGetLastError();
}

hipError_t fl_weights(hipStream_t s, int64_t n, const double* logtheta, const WeightArgs& a, double* W, int64_t ldw) {
    if (n <= 0 || a.count <= 0) return hipSuccess;
    dim3 grid((unsigned)FL_DIV_UP(n, 256), (unsigned)a.count);
    weights_kernel<<<grid, 256, 0, s>>>(n, logtheta, a, W, ldw);
    return hipGetLastError();
}

namespace {
template <class BS>
hipError_t scaled_launch(hipStream_t s, dim3 grid, int64_t n, int64_t ncol, const double* V, int64_t ldv,
                         const BS& bs, double* U, int64_t ldu, const GemmChoice& c) {
    const int64_t group = c.group > 0 ? c.group : 8;
    if (c.variant == FL_GV_SQUARE32)
        scaled_gemm_kernel<BS, 32><<<grid, NT, 0, s>>>(n, ncol, V, ldv, bs, U, ldu, group);
    else
        scaled_gemm_kernel<BS, 16><<<grid, NT, 0, s>>>(n, ncol, V, ldv, bs, U, ldu, group);
    return hipGetLastError();
}
}  // namespace

hipError_t fl_scaled_gemm(hipStream_t s, int64_t n, const double* V, int64_t ldv, const double* W, int64_t ldw,
                          const double* C, int64_t ldc, int64_t nf, int64_t na, int paired, double* U,
                          int64_t ldu, const GemmChoice* forced, bool timed) {
    int64_t ncol = paired ? nf : nf * na;
    if (n <= 0 || ncol <= 0) return hipSuccess;
    dim3 grid((unsigned)FL_DIV_UP(n, BM), (unsigned)FL_DIV_UP(ncol, BN));
    const GemmChoice c = forced ? *forced : tuned_choice(FL_TUNE_SCALED, 0, 0, n, ncol, n);
    KScope ks(timed ? "scaled_gemm" : nullptr, s);
    if (!paired && nf % BN == 0) {
        BScaledUniform bs{W, ldw, C, ldc, nf};
        return scaled_launch(s, grid, n, ncol, V, ldv, bs, U, ldu, c);
    }
    BScaled bs{W, ldw, C, ldc, nf, paired};
    return scaled_launch(s, grid, n, ncol, V, ldv, bs, U, ldu, c);
}

hipError_t fl_spec_grad(hipStream_t s, int64_t n, const double* P, int64_t ldp, const double* C, int64_t ldc,
                        const double* W, int64_t ldw, const double* logtheta, const WeightArgs& a, double* ga,
                        double* gs) {
    if (a.count <= 0) return hipSuccess;
    spec_grad_kernel<<<(unsigned)a.count, 256, 0, s>>>(n, P, ldp, C, ldc, W, ldw, logtheta, a, ga, gs);
    return hipGetLastError();
}

hipError_t fl_check_finite(hipStream_t s, int64_t m, int64_t n, const double* A, int64_t lda, int* flag) {
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 grid((unsigned)FL_DIV_UP(m, 256), (unsigned)(n < 65535 ? n : 65535));
    finite_kernel<<<grid, 256, 0, s>>>(m, n, A, lda, flag);
    return hipGetLastError();
}
