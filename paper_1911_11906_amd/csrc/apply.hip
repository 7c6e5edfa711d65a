// Spectral application v = sum_k theta_k^(-alpha/2) (phi_k^T M f) phi_k
// (Section "Method", equations for g and v) and its adjoint.
//
//   G = M F            CSR SpMM (HBM bound)
//   C = V^T G          FP64 MFMA GEMM
//   W_ki = exp(-(alpha_i/2) ln theta_k)       (alpha = 0 gives exactly 1)
//   U[:, j + i nf] = V (W[:, i] o C[:, j])    one FP64 MFMA GEMM whose
//        operand B is formed while it is staged into LDS, so the
//        na-times-larger scaled operand never exists in memory.
// Adjoint (paired pairs b): P = V^T GU,
//   galpha_b = sum_k P_kb (-ln(theta_k)/2) W_kb C_kb,   GF = M V (W o P).
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

__global__ void weights_kernel(int64_t n, const double* __restrict__ logtheta, int64_t na,
                               const double* __restrict__ alpha, double* __restrict__ W, int64_t ldw) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double lt = logtheta[k];
    for (int64_t i = blockIdx.y; i < na; i += gridDim.y) W[k + i * ldw] = exp(-0.5 * alpha[i] * lt);
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

template <class BS>
__global__ __launch_bounds__(NT) FL_TWO_WAVES_PER_SIMD void scaled_gemm_kernel(int64_t n, int64_t ncol, const double* __restrict__ V,
                                                         int64_t ldv, BS bs, double* __restrict__ U,
                                                         int64_t ldu) {
    __shared__ double As[TileLds<16, 1>::A];
    __shared__ double Bs[TileLds<16, 1>::B];
    int64_t bi, bj;
    xcd_grouped_tile(bi, bj);
    tile_gemm<false, true, BS, 16, 1>(n, ncol, n, V, ldv, bs, 1.0, 0.0, U, ldu, bi, bj, As, Bs);
}

// galpha[b] = sum_k P[k,b] * (-0.5 ln theta_k) * W[k,b] * C[k,b]; one block per b,
// fixed-order tree reduction (deterministic).
__global__ __launch_bounds__(256) void galpha_kernel(int64_t n, const double* __restrict__ P, int64_t ldp,
                                                     const double* __restrict__ C, int64_t ldc,
                                                     const double* __restrict__ W, int64_t ldw,
                                                     const double* __restrict__ logtheta, double* out) {
    __shared__ double red[256];
    int64_t b = blockIdx.x;
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += 256)
        s += P[k + b * ldp] * (-0.5 * logtheta[k]) * W[k + b * ldw] * C[k + b * ldc];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[b] = red[0];
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

hipError_t fl_weights(hipStream_t s, int64_t n, const double* logtheta, int64_t na, const double* alpha,
                      double* W, int64_t ldw) {
    if (n <= 0 || na <= 0) return hipSuccess;
    dim3 grid((unsigned)FL_DIV_UP(n, 256), (unsigned)(na < 65535 ? na : 65535));
    weights_kernel<<<grid, 256, 0, s>>>(n, logtheta, na, alpha, W, ldw);
    return hipGetLastError();
}

hipError_t fl_scaled_gemm(hipStream_t s, int64_t n, const double* V, int64_t ldv, const double* W, int64_t ldw,
                          const double* C, int64_t ldc, int64_t nf, int64_t na, int paired, double* U,
                          int64_t ldu) {
    int64_t ncol = paired ? nf : nf * na;
    if (n <= 0 || ncol <= 0) return hipSuccess;
    dim3 grid((unsigned)FL_DIV_UP(n, BM), (unsigned)FL_DIV_UP(ncol, BN));
    KScope ks("scaled_gemm", s);
    if (!paired && nf % BN == 0) {
        BScaledUniform bs{W, ldw, C, ldc, nf};
        scaled_gemm_kernel<BScaledUniform><<<grid, NT, 0, s>>>(n, ncol, V, ldv, bs, U, ldu);
    } else {
        BScaled bs{W, ldw, C, ldc, nf, paired};
        scaled_gemm_kernel<BScaled><<<grid, NT, 0, s>>>(n, ncol, V, ldv, bs, U, ldu);
    }
    return hipGetLastError();
}

hipError_t fl_galpha(hipStream_t s, int64_t n, int64_t nb, const double* P, int64_t ldp, const double* C,
                     int64_t ldc, const double* W, int64_t ldw, const double* logtheta, double* out) {
    if (nb <= 0) return hipSuccess;
    galpha_kernel<<<(unsigned)nb, 256, 0, s>>>(n, P, ldp, C, ldc, W, ldw, logtheta, out);
    return hipGetLastError();
}

hipError_t fl_check_finite(hipStream_t s, int64_t m, int64_t n, const double* A, int64_t lda, int* flag) {
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 grid((unsigned)FL_DIV_UP(m, 256), (unsigned)(n < 65535 ? n : 65535));
    finite_kernel<<<grid, 256, 0, s>>>(m, n, A, lda, flag);
    return hipGetLastError();
}
