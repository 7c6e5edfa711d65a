// FP64 MFMA GEMM tile machinery shared by the plain GEMM and the fused
// spectral-application GEMM (operand B produced on the fly).
//
// v_mfma_f64_16x16x4f64 operand layout (measured on gfx950): lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; accumulator register r of lane l holds
// D[l/16 + 4r][l%16].  We compute C^T tiles (MFMA "A" <- op(B), "B" <- op(A))
// so that lanes sharing an accumulator row write consecutive rows of the
// column-major C.  Workgroup tile 128 x 128, k-step 16, 256 threads as 2 x 2
// waves of 64 x 64, operands staged k-major in LDS and double buffered.
#pragma once
#include "common.h"

namespace fl_tile {

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int SA = BM + 2;  // LDS row strides (doubles)
constexpr int SB = BN + 2;
constexpr int NT = 256;
// LDS doubles needed by tile_gemm<.., KB, NBUF>
template <int KB, int NBUF>
struct TileLds {
    static constexpr int A = NBUF * KB * SA;
    static constexpr int B = NBUF * KB * SB;
};

// Source of op(B)[kk][j].  A thread's columns j are fixed for the whole k
// loop, so each source hands out a per-column handle once (col()) and then
// reads element kk through it (at()).
struct BPlain {
    const double* B;
    int64_t ldb;
    bool trans;
    struct H {
        const double* p;
        int64_t stride;
    };
    __device__ inline H col(int64_t j) const { return trans ? H{B + j, ldb} : H{B + j * ldb, 1}; }
    __device__ inline double at(const H& h, int64_t kk) const { return h.p[kk * h.stride]; }
    // per-(tile, k-row) factor applied to every element of that k-row
    static constexpr bool KSCALE = false;
    __device__ inline double kscale(int64_t, int64_t) const { return 1.0; }
};

// KB: k-step; NBUF: LDS buffers (2 = double buffered, one barrier per step;
// 1 = register prefetch, two barriers per step, half the LDS).
template <bool TA, bool KFAST_B, class BSrc, int KB = 32, int NBUF = 1>
__device__ inline void tile_gemm(int64_t m, int64_t n, int64_t k, const double* __restrict__ A, int64_t lda,
                                 const BSrc& bs, double alpha, double beta, double* __restrict__ C, int64_t ldc,
                                 int64_t bi, int64_t bj, double* As, double* Bs) {
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wi = wave & 1, wj = wave >> 1;
    const int64_t i0 = bi * BM, j0 = bj * BN;
    d4_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
    constexpr int NA = BM * KB / NT, NB = BN * KB / NT;
    double ra[NA], rb[NB];
    typename BSrc::H bh[NB];
    bool bok[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        int e = t + NT * r;
        int jj = KFAST_B ? e / KB : e % BN;
        int64_t gj = j0 + jj;
        bok[r] = gj < n;
        bh[r] = bs.col(bok[r] ? gj : j0);
    }
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            int e = t + NT * r;
            int ii, kk;
            if (!TA) { ii = e % BM; kk = e / BM; } else { kk = e % KB; ii = e / KB; }
            int64_t gi = i0 + ii, gk = k0 + kk;
            double v = 0.0;
            if (gi < m && gk < k) v = TA ? A[gk + gi * lda] : A[gi + gk * lda];
            ra[r] = v;
        }
        // with KFAST_B every element a thread loads shares one k-row (t % KB)
        double ks = 1.0;
        if (BSrc::KSCALE && KFAST_B && k0 + (t % KB) < k) ks = bs.kscale(j0, k0 + (t % KB));
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            int e = t + NT * r;
            int jj, kk;
            if (KFAST_B) { kk = e % KB; jj = e / KB; } else { jj = e % BN; kk = e / BN; }
            int64_t gk = k0 + kk;
            (void)jj;
            double v = (bok[r] && gk < k) ? bs.at(bh[r], gk) : 0.0;
            rb[r] = BSrc::KSCALE ? v * ks : v;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            int e = t + NT * r;
            int ii, kk;
            if (!TA) { ii = e % BM; kk = e / BM; } else { kk = e % KB; ii = e / KB; }
            As[buf * KB * SA + kk * SA + ii] = ra[r];
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            int e = t + NT * r;
            int jj, kk;
            if (KFAST_B) { kk = e % KB; jj = e / KB; } else { jj = e % BN; kk = e / BN; }
            Bs[buf * KB * SB + kk * SB + jj] = rb[r];
        }
    };
    const int64_t nkt = FL_DIV_UP(k, KB);
    const int lr = lane >> 4, lc = lane & 15;
    auto compute = [&](const double* Ac, const double* Bc) {
#pragma unroll
        for (int k4 = 0; k4 < KB; k4 += 4) {
            double fa[4], fb[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                fa[q] = Bc[(k4 + lr) * SB + wj * 64 + q * 16 + lc];  // MFMA A operand <- op(B)
                fb[q] = Ac[(k4 + lr) * SA + wi * 64 + q * 16 + lc];  // MFMA B operand <- op(A)
            }
#pragma unroll
            for (int ib = 0; ib < 4; ++ib)
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
                    acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[jb], fb[ib], acc[ib][jb], 0, 0, 0);
        }
    };
    if (NBUF == 2) {
        if (nkt > 0) {
            gload(0);
            sstore(0);
        }
        __syncthreads();
        for (int64_t kt = 0; kt < nkt; ++kt) {
            const int cur = (int)(kt & 1);
            if (kt + 1 < nkt) gload((kt + 1) * KB);
            compute(As + cur * KB * SA, Bs + cur * KB * SB);
            if (kt + 1 < nkt) sstore(1 - cur);
            __syncthreads();
        }
    } else {
        if (nkt > 0) gload(0);
        for (int64_t kt = 0; kt < nkt; ++kt) {
            __syncthreads();
            sstore(0);
            __syncthreads();
            if (kt + 1 < nkt) gload((kt + 1) * KB);
            compute(As, Bs);
        }
    }
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) {
        int64_t gi = i0 + wi * 64 + ib * 16 + lc;
        if (gi >= m) continue;
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int64_t gj = j0 + wj * 64 + jb * 16 + lr + 4 * r;
                if (gj >= n) continue;
                double* cp = C + gi + gj * ldc;
                double v = alpha * acc[ib][jb][r];
                if (beta != 0.0) v += beta * (*cp);
                *cp = v;
            }
        }
    }
}

}  // namespace fl_tile
