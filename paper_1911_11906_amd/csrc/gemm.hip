// Dense GEMM on the CDNA4 matrix cores (tile machinery in gemm_tile.h).
//
// FP64: v_mfma_f64_16x16x4f64.  Operand layout (measured on gfx950): lane l
// supplies A[l%16][l/16] and B[l/16][l%16]; the 4 accumulator registers of
// lane l hold D[l/16 + 4r][l%16], r = 0..3.
// FP32: v_mfma_f32_16x16x4f32, same inputs, accumulator D[4(l/16) + r][l%16].
//
// We compute C^T tiles: the MFMA "A" operand is fed from op(B) and the "B"
// operand from op(A), so the 16 lanes that share an accumulator row write 16
// consecutive rows of the column-major C (128-byte segments).
//
// Workgroup tile 128 x 128, k-step 16, 256 threads = 2 x 2 waves of 64 x 64.
// Both operand tiles are staged k-major in LDS and double buffered; one
// barrier per k-step.
#include <algorithm>
#include "gemm_tile.h"

namespace {
using namespace fl_tile;

constexpr int GKB = 32, GNBUF = 1;  // k-step 32 with register prefetch (measured best on gfx950)

template <bool TA, bool TB, bool LOWER>
__global__ __launch_bounds__(NT) void dgemm_kernel(GemmProblem g) {
    __shared__ double As[TileLds<GKB, GNBUF>::A];
    __shared__ double Bs[TileLds<GKB, GNBUF>::B];
    const int64_t bi = blockIdx.x, bj = blockIdx.y;
    if (LOWER && (bi + 1) * BM <= bj * BN) return;  // tile strictly above the diagonal
    BPlain bsrc{g.B, g.ldb, TB};
    tile_gemm<TA, !TB, BPlain, GKB, GNBUF>(g.m, g.n, g.k, g.A, g.lda, bsrc, g.alpha, g.beta, g.C, g.ldc, bi, bj, As,
                                           Bs);
}

// Split-K: slice z of the k range into its own partial product P_z (beta = 0).
template <bool TA, bool TB>
__global__ __launch_bounds__(NT) void dgemm_splitk_kernel(GemmProblem g, int64_t kc, double* P) {
    __shared__ double As[TileLds<GKB, GNBUF>::A];
    __shared__ double Bs[TileLds<GKB, GNBUF>::B];
    const int64_t z = blockIdx.z;
    const int64_t koff = z * kc;
    const int64_t ks = (g.k - koff) < kc ? (g.k - koff) : kc;
    const double* A = TA ? g.A + koff : g.A + koff * g.lda;
    const double* B = TB ? g.B + koff * g.ldb : g.B + koff;
    BPlain bsrc{B, g.ldb, TB};
    tile_gemm<TA, !TB, BPlain, GKB, GNBUF>(g.m, g.n, ks > 0 ? ks : 0, A, g.lda, bsrc, g.alpha, 0.0, P + z * g.m * g.n,
                                           g.m, blockIdx.x, blockIdx.y, As, Bs);
}

// C = beta C + sum_z P_z, fixed summation order (deterministic)
__global__ void splitk_reduce_kernel(int64_t m, int64_t n, int S, const double* __restrict__ P, double beta,
                                     double* C, int64_t ldc) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
        double acc = 0.0;
        for (int z = 0; z < S; ++z) acc += P[(int64_t)z * m * n + i + j * m];
        double* c = C + i + j * ldc;
        *c = (beta != 0.0) ? beta * (*c) + acc : acc;
    }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(NT) void dgemm_batched_kernel(const GemmProblem* __restrict__ probs) {
    __shared__ double As[TileLds<GKB, GNBUF>::A];
    __shared__ double Bs[TileLds<GKB, GNBUF>::B];
    const GemmProblem g = probs[blockIdx.z];
    const int64_t bi = blockIdx.x, bj = blockIdx.y;
    if (bi * BM >= g.m || bj * BN >= g.n) return;
    BPlain bsrc{g.B, g.ldb, TB};
    tile_gemm<TA, !TB, BPlain, GKB, GNBUF>(g.m, g.n, g.k, g.A, g.lda, bsrc, g.alpha, g.beta, g.C, g.ldc, bi, bj, As,
                                           Bs);
}

// Split-K workspace: one buffer per device, allocated once and never resized
// (a resize could free memory that queued kernels still use); the split
// factor is capped to what fits.
constexpr int64_t SPLITK_WS = 32ll << 20;  // doubles (256 MB)
double* splitk_ws(int dev) {
    static double* ws[64] = {nullptr};
    static bool failed[64] = {false};
    if (dev < 0 || dev >= 64) return nullptr;
    if (!ws[dev] && !failed[dev]) {
        if (hipMalloc(&ws[dev], sizeof(double) * SPLITK_WS) != hipSuccess) {
            ws[dev] = nullptr;
            failed[dev] = true;
            (void)hipGetLastError();
        }
    }
    return ws[dev];
}

template <bool TA, bool TB>
hipError_t launch(hipStream_t s, const GemmProblem& g, int lower) {
    const int64_t tm = FL_DIV_UP(g.m, BM), tn = FL_DIV_UP(g.n, BN);
    const int64_t tiles = tm * tn;
    // few output tiles and a long k: split k so that the chip fills up
    if (!lower && tiles < 384 && g.k >= 2048) {
        int64_t S = std::min<int64_t>({FL_DIV_UP(768, tiles), g.k / 512, 32});
        while (S > 1 && S * g.m * g.n > SPLITK_WS) --S;
        int dev = 0;
        double* P = (S > 1 && hipGetDevice(&dev) == hipSuccess) ? splitk_ws(dev) : nullptr;
        if (S > 1 && P) {
            int64_t kc = FL_DIV_UP(FL_DIV_UP(g.k, S), GKB) * GKB;
            S = FL_DIV_UP(g.k, kc);
            dgemm_splitk_kernel<TA, TB><<<dim3((unsigned)tm, (unsigned)tn, (unsigned)S), NT, 0, s>>>(g, kc, P);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            dim3 rg((unsigned)FL_DIV_UP(g.m, 256), (unsigned)std::min<int64_t>(g.n, 65535));
            splitk_reduce_kernel<<<rg, 256, 0, s>>>(g.m, g.n, (int)S, P, g.beta, g.C, g.ldc);
            return hipGetLastError();
        }
    }
    dim3 grid((unsigned)tm, (unsigned)tn);
    if (lower)
        dgemm_kernel<TA, TB, true><<<grid, NT, 0, s>>>(g);
    else
        dgemm_kernel<TA, TB, false><<<grid, NT, 0, s>>>(g);
    return hipGetLastError();
}

// ---------------------------------------------------------------- FP32
constexpr int SBM = 128, SBN = 128, SBK = 32;
constexpr int SSA = SBM + 4, SSB = SBN + 4;

template <bool TA, bool TB>
__global__ __launch_bounds__(NT) void sgemm_kernel(int64_t m, int64_t n, int64_t k, float alpha,
                                                   const float* __restrict__ A, int64_t lda,
                                                   const float* __restrict__ B, int64_t ldb, float beta,
                                                   float* __restrict__ C, int64_t ldc) {
    __shared__ float As[2 * SBK * SSA];
    __shared__ float Bs[2 * SBK * SSB];
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wi = wave & 1, wj = wave >> 1;
    const int64_t i0 = (int64_t)blockIdx.x * SBM, j0 = (int64_t)blockIdx.y * SBN;
    f4_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f4_t{0.f, 0.f, 0.f, 0.f};
    constexpr int NA = SBM * SBK / NT, NB = SBN * SBK / NT;
    float ra[NA], rb[NB];
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            int e = t + NT * r;
            int ii, kk;
            if (!TA) { ii = e % SBM; kk = e / SBM; } else { kk = e % SBK; ii = e / SBK; }
            int64_t gi = i0 + ii, gk = k0 + kk;
            ra[r] = (gi < m && gk < k) ? (TA ? A[gk + gi * lda] : A[gi + gk * lda]) : 0.f;
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            int e = t + NT * r;
            int jj, kk;
            if (!TB) { kk = e % SBK; jj = e / SBK; } else { jj = e % SBN; kk = e / SBN; }
            int64_t gj = j0 + jj, gk = k0 + kk;
            rb[r] = (gj < n && gk < k) ? (TB ? B[gj + gk * ldb] : B[gk + gj * ldb]) : 0.f;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            int e = t + NT * r;
            int ii, kk;
            if (!TA) { ii = e % SBM; kk = e / SBM; } else { kk = e % SBK; ii = e / SBK; }
            As[buf * SBK * SSA + kk * SSA + ii] = ra[r];
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            int e = t + NT * r;
            int jj, kk;
            if (!TB) { kk = e % SBK; jj = e / SBK; } else { jj = e % SBN; kk = e / SBN; }
            Bs[buf * SBK * SSB + kk * SSB + jj] = rb[r];
        }
    };
    const int64_t nkt = FL_DIV_UP(k, SBK);
    if (nkt > 0) { gload(0); sstore(0); }
    __syncthreads();
    const int lr = lane >> 4, lc = lane & 15;
    for (int64_t kt = 0; kt < nkt; ++kt) {
        const int cur = (int)(kt & 1);
        if (kt + 1 < nkt) gload((kt + 1) * SBK);
        const float* Ac = As + cur * SBK * SSA;
        const float* Bc = Bs + cur * SBK * SSB;
#pragma unroll
        for (int k4 = 0; k4 < SBK; k4 += 4) {
            float fa[4], fb[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                fa[q] = Bc[(k4 + lr) * SSB + wj * 64 + q * 16 + lc];
                fb[q] = Ac[(k4 + lr) * SSA + wi * 64 + q * 16 + lc];
            }
#pragma unroll
            for (int ib = 0; ib < 4; ++ib)
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
                    acc[ib][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[jb], fb[ib], acc[ib][jb], 0, 0, 0);
        }
        if (kt + 1 < nkt) sstore(1 - cur);
        __syncthreads();
    }
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) {
        int64_t gi = i0 + wi * 64 + ib * 16 + lc;
        if (gi >= m) continue;
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int64_t gj = j0 + wj * 64 + jb * 16 + 4 * lr + r;  // FP32 layout: D[4(l/16)+r][l%16]
                if (gj >= n) continue;
                float* cp = C + gi + gj * ldc;
                float v = alpha * acc[ib][jb][r];
                if (beta != 0.f) v += beta * (*cp);
                *cp = v;
            }
    }
}

// ---------------------------------------------------------------- helpers
__global__ void copy_kernel(int64_t m, int64_t n, const double* __restrict__ A, int64_t lda,
                            double* __restrict__ B, int64_t ldb) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t j = blockIdx.y;
    for (; j < n; j += gridDim.y)
        if (i < m) B[i + j * ldb] = A[i + j * lda];
}

__global__ void transpose_kernel(int64_t m, int64_t n, const double* __restrict__ A, int64_t lda,
                                 double* __restrict__ B, int64_t ldb) {
    __shared__ double tile[32][33];
    int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
    int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        int64_t i = i0 + tx, j = j0 + r;
        if (i < m && j < n) tile[r][tx] = A[i + j * lda];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        int64_t jj = j0 + tx, ii = i0 + r;  // B(j, i) = A(i, j)
        if (ii < m && jj < n) B[jj + ii * ldb] = tile[tx][r];
    }
}

__global__ void fill_kernel(int64_t m, int64_t n, double v, double* A, int64_t lda) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        if (i < m) A[i + j * lda] = v;
}

__global__ void identity_kernel(int64_t n, double* A, int64_t lda) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        if (i < n) A[i + j * lda] = (i == j) ? 1.0 : 0.0;
}

inline dim3 grid2(int64_t m, int64_t n) {
    int64_t gy = n < 65535 ? n : 65535;
    return dim3((unsigned)FL_DIV_UP(m, 256), (unsigned)(gy > 0 ? gy : 1));
}

}  // namespace

hipError_t fl_dgemm(hipStream_t s, int ta, int tb, int64_t m, int64_t n, int64_t k, double alpha,
                    const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                    int64_t ldc, int lower) {
    if (m <= 0 || n <= 0) return hipSuccess;
    if (k <= 0 && beta == 1.0) return hipSuccess;
    GemmProblem g{m, n, k, A, lda, B, ldb, C, ldc, alpha, beta};
    if (!ta && !tb) return launch<false, false>(s, g, lower);
    if (!ta && tb) return launch<false, true>(s, g, lower);
    if (ta && !tb) return launch<true, false>(s, g, lower);
    return launch<true, true>(s, g, lower);
}

hipError_t fl_dgemm_batched(hipStream_t s, int ta, int tb, const GemmProblem* probs, int count, int64_t max_m,
                            int64_t max_n) {
    if (count <= 0 || max_m <= 0 || max_n <= 0) return hipSuccess;
    dim3 grid((unsigned)FL_DIV_UP(max_m, BM), (unsigned)FL_DIV_UP(max_n, BN), (unsigned)count);
    if (!ta && !tb)
        dgemm_batched_kernel<false, false><<<grid, NT, 0, s>>>(probs);
    else if (!ta && tb)
        dgemm_batched_kernel<false, true><<<grid, NT, 0, s>>>(probs);
    else if (ta && !tb)
        dgemm_batched_kernel<true, false><<<grid, NT, 0, s>>>(probs);
    else
        dgemm_batched_kernel<true, true><<<grid, NT, 0, s>>>(probs);
    return hipGetLastError();
}

hipError_t fl_sgemm(hipStream_t s, int ta, int tb, int64_t m, int64_t n, int64_t k, float alpha, const float* A,
                    int64_t lda, const float* B, int64_t ldb, float beta, float* C, int64_t ldc) {
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 grid((unsigned)FL_DIV_UP(m, SBM), (unsigned)FL_DIV_UP(n, SBN));
    if (!ta && !tb)
        sgemm_kernel<false, false><<<grid, NT, 0, s>>>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
    else if (!ta && tb)
        sgemm_kernel<false, true><<<grid, NT, 0, s>>>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
    else if (ta && !tb)
        sgemm_kernel<true, false><<<grid, NT, 0, s>>>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
    else
        sgemm_kernel<true, true><<<grid, NT, 0, s>>>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
    return hipGetLastError();
}

hipError_t fl_copy_matrix(hipStream_t s, int64_t m, int64_t n, const double* A, int64_t lda, double* B,
                          int64_t ldb) {
    if (m <= 0 || n <= 0) return hipSuccess;
    copy_kernel<<<grid2(m, n), 256, 0, s>>>(m, n, A, lda, B, ldb);
    return hipGetLastError();
}

hipError_t fl_transpose(hipStream_t s, int64_t m, int64_t n, const double* A, int64_t lda, double* B,
                        int64_t ldb) {
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 grid((unsigned)FL_DIV_UP(m, 32), (unsigned)FL_DIV_UP(n, 32));
    transpose_kernel<<<grid, dim3(32, 8), 0, s>>>(m, n, A, lda, B, ldb);
    return hipGetLastError();
}

hipError_t fl_fill(hipStream_t s, int64_t m, int64_t n, double v, double* A, int64_t lda) {
    if (m <= 0 || n <= 0) return hipSuccess;
    fill_kernel<<<grid2(m, n), 256, 0, s>>>(m, n, v, A, lda);
    return hipGetLastError();
}

hipError_t fl_set_identity(hipStream_t s, int64_t n, double* A, int64_t lda) {
    if (n <= 0) return hipSuccess;
    identity_kernel<<<grid2(n, n), 256, 0, s>>>(n, A, lda);
    return hipGetLastError();
}
