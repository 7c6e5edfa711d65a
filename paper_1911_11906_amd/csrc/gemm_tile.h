// FP64 / FP32 MFMA GEMM tile machinery shared by the plain GEMMs and the
// fused spectral-application GEMM (operand B produced on the fly).
//
// v_mfma_f64_16x16x4f64 operand layout (measured on gfx950): lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; accumulator register r of lane l holds
// D[l/16 + 4r][l%16].  We compute C^T tiles (MFMA "A" <- op(B), "B" <- op(A))
// so that lanes sharing an accumulator row write consecutive rows of the
// column-major C.  Workgroup tile 128 x 128 (or 256 x 64), 256 threads as
// four waves of 64 x 64, operands staged k-major in LDS; the next k-step's
// operands are prefetched into registers (NBUF = 1) or a second LDS buffer
// (NBUF = 2) while the current one is multiplied.
#pragma once
#include "common.h"
#include <type_traits>

namespace fl_tile {

// Matrix-core instruction per element type.  FP64: v_mfma_f64_16x16x4f64,
// accumulator register r of lane l holds D[l/16 + 4r][l%16]; FP32:
// v_mfma_f32_16x16x4f32, D[4(l/16) + r][l%16].  Inputs: lane l supplies
// A[l%16][l/16] and B[l/16][l%16] for both.
template <class T> struct Mfma;
template <> struct Mfma<double> {
    typedef d4_t acc;
    static __device__ inline acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lr, int r) { return lr + 4 * r; }
};
template <> struct Mfma<float> {
    typedef f4_t acc;
    static __device__ inline acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lr, int r) { return 4 * lr + r; }
};

// Tile kernels are compiled for two waves per SIMD (at most 256 registers per
// lane, accumulators included), so two workgroups share a CU and one's LDS
// staging and barriers overlap the other's matrix-core work.
#define FL_TWO_WAVES_PER_SIMD __attribute__((amdgpu_waves_per_eu(2, 2)))

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int SA = BM + 2;  // LDS row strides (doubles)
constexpr int SB = BN + 2;
constexpr int NT = 256;
// Tile coordinates of a full (tm x tn) grid in an XCD-aware grouped order.
// Consecutive workgroup ids go to the eight XCDs in turn, so id is first
// split into (id mod 8, id / 8) and each XCD gets one contiguous eighth of
// the grouped order (when the tile count is a multiple of 8); that order
// walks bands of GM row tiles column by column, so the workgroups resident
// on one XCD at a time cover a compact GM x (resident / GM) patch and share
// its row and column blocks in that XCD's L2.  A bijection of the grid.
__device__ inline void xcd_grouped_tile(int64_t& bi, int64_t& bj, int64_t GM = 8) {
    const int64_t tm = gridDim.x, tn = gridDim.y, T = tm * tn;
    const int64_t id = blockIdx.x + tm * (int64_t)blockIdx.y;
    const int64_t L = (T % 8 == 0) ? (id % 8) * (T / 8) + id / 8 : id;
    const int64_t g = L / (GM * tn);
    const int64_t rows = (tm - g * GM < GM) ? tm - g * GM : GM;
    const int64_t q = L - g * GM * tn;
    bi = g * GM + q % rows;
    bj = q / rows;
}

// LDS doubles needed by tile_gemm<.., KB, NBUF, T, WM>: WM waves along M
// (workgroup tile 64 WM x 64 (4 / WM); WM = 2: 128 x 128, WM = 4: 256 x 64
// for products with at most 64 columns)
template <int KB, int NBUF, int WM = 2>
struct TileLds {
    static constexpr int A = NBUF * KB * (64 * WM + 2);
    static constexpr int B = NBUF * KB * (64 * (4 / WM) + 2);
};
// (elements of the tile's element type)

// Source of op(B)[kk][j].  A thread's columns j are fixed for the whole k
// loop, so each source hands out a per-column handle once (col()) and then
// reads element kk through it (at()).
template <class T>
struct BPlainT {
    const T* B;
    int64_t ldb;
    bool trans;
    struct H {
        const T* p;
        int64_t stride;
    };
    __device__ inline H col(int64_t j) const { return trans ? H{B + j, ldb} : H{B + j * ldb, 1}; }
    __device__ inline T at(const H& h, int64_t kk) const { return h.p[kk * h.stride]; }
    // per-(tile, k-row) factor applied to every element of that k-row:
    // kcol(first column of the tile) once per tile, then kscale(kcol, k)
    static constexpr bool KSCALE = false;
    __device__ inline const T* kcol(int64_t) const { return nullptr; }
    __device__ inline T kscale(const T*, int64_t) const { return T(1); }
};
typedef BPlainT<double> BPlain;

// KB: k-step; NBUF: LDS buffers (2 = double buffered, one barrier per step;
// 1 = register prefetch, two barriers per step, half the LDS).
template <bool TA, bool KFAST_B, class BSrc, int KB = 32, int NBUF = 1, class T = double, int WM = 2>
__device__ inline void tile_gemm(int64_t m, int64_t n, int64_t k, const T* __restrict__ A, int64_t lda,
                                 const BSrc& bs, T alpha, T beta, T* __restrict__ C, int64_t ldc,
                                 int64_t bi, int64_t bj, T* As, T* Bs) {
    typedef typename Mfma<T>::acc acc_t;
    constexpr int BM = 64 * WM, BN = 64 * (4 / WM), SA = BM + 2, SB = BN + 2;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wi = wave % WM, wj = wave / WM;
    const int64_t i0 = bi * BM, j0 = bj * BN;
    acc_t acc[4][4];
    // beta = +-1 with alpha = +-1: C (times beta / alpha, exact) is loaded into
    // the accumulators before the k loop, so that its read overlaps the first
    // operand loads instead of following the last product
    const bool pre = (beta == T(1) || beta == T(-1)) && (alpha == T(1) || alpha == T(-1));
    {
        const int plr = (t & 63) >> 4, plc = t & 15;
        const T f = beta * alpha;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int64_t gi = i0 + wi * 64 + a * 16 + plc;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                acc[a][b] = acc_t{0, 0, 0, 0};
                if (pre && gi < m) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t gj = j0 + wj * 64 + b * 16 + Mfma<T>::row(plr, r);
                        if (gj < n) acc[a][b][r] = f * C[gi + gj * ldc];
                    }
                }
            }
        }
    }
    constexpr int NA = BM * KB / NT, NB = BN * KB / NT;
    T ra[NA], rb[NB];
    typename BSrc::H bh[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        int e = t + NT * r;
        int jj = KFAST_B ? e / KB : e % BN;
        int64_t gj = j0 + jj;
        bh[r] = bs.col(gj < n ? gj : n - 1);
    }
    // Operand loads are unconditional: rows of A beyond m and columns of B
    // beyond n read a clamped, valid row / column (their products land in
    // outputs that are never stored); only a partial last k-step clamps k and
    // writes zeros for the rows past k.  No load sits in a branch, so the
    // compiler need not wait for one before the next.
    const auto kc = bs.kcol(j0);  // per-tile k-row factors (KSCALE sources)
    auto gload = [&](int64_t k0, auto edge) {
        constexpr bool EDGE = decltype(edge)::value;
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            int e = t + NT * r;
            int ii, kk;
            if (!TA) { ii = e % BM; kk = e / BM; } else { kk = e % KB; ii = e / KB; }
            int64_t gi = i0 + ii, gk = k0 + kk;
            gi = gi < m ? gi : m - 1;
            if (EDGE) gk = gk < k ? gk : k - 1;
            ra[r] = TA ? A[gk + gi * lda] : A[gi + gk * lda];
        }
        // with KFAST_B every element a thread loads shares one k-row (t % KB)
        T ks = T(1);
        if (BSrc::KSCALE && KFAST_B) {
            int64_t gk = k0 + (t % KB);
            if (EDGE) gk = gk < k ? gk : k - 1;
            ks = bs.kscale(kc, gk);
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            int e = t + NT * r;
            int kk = KFAST_B ? e % KB : e / BN;
            int64_t gk = k0 + kk;
            if (EDGE) gk = gk < k ? gk : k - 1;
            T v = bs.at(bh[r], gk);
            rb[r] = BSrc::KSCALE ? v * ks : v;
        }
    };
    auto sstore = [&](int buf, int64_t k0, auto edge) {
        constexpr bool EDGE = decltype(edge)::value;
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            int e = t + NT * r;
            int ii, kk;
            if (!TA) { ii = e % BM; kk = e / BM; } else { kk = e % KB; ii = e / KB; }
            As[buf * KB * SA + kk * SA + ii] = (EDGE && k0 + kk >= k) ? T(0) : ra[r];
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            int e = t + NT * r;
            int jj, kk;
            if (KFAST_B) { kk = e % KB; jj = e / KB; } else { jj = e % BN; kk = e / BN; }
            Bs[buf * KB * SB + kk * SB + jj] = (EDGE && k0 + kk >= k) ? T(0) : rb[r];
        }
    };
    const int64_t nkt = FL_DIV_UP(k, KB);
    const int lr = lane >> 4, lc = lane & 15;
    auto compute = [&](const T* Ac, const T* Bc) {
#pragma unroll
        for (int k4 = 0; k4 < KB; k4 += 4) {
            T fa[4], fb[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                fa[q] = Bc[(k4 + lr) * SB + wj * 64 + q * 16 + lc];  // MFMA A operand <- op(B)
                fb[q] = Ac[(k4 + lr) * SA + wi * 64 + q * 16 + lc];  // MFMA B operand <- op(A)
            }
#pragma unroll
            for (int ib = 0; ib < 4; ++ib)
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
                    acc[ib][jb] = Mfma<T>::mma(fa[jb], fb[ib], acc[ib][jb]);
        }
    };
    // k-step kt is partial only when it is the last one and KB does not divide k
    const bool kpart = (k % KB) != 0;
    auto is_edge = [&](int64_t kt) { return kpart && kt == nkt - 1; };
    const std::true_type E1;
    const std::false_type E0;
    if (NBUF == 2) {
        if (nkt > 0) {
            if (is_edge(0)) { gload(0, E1); sstore(0, 0, E1); }
            else { gload(0, E0); sstore(0, 0, E0); }
        }
        __syncthreads();
        for (int64_t kt = 0; kt < nkt; ++kt) {
            const int cur = (int)(kt & 1);
            const bool nedge = is_edge(kt + 1);
            if (kt + 1 < nkt) {
                if (nedge) gload((kt + 1) * KB, E1);
                else gload((kt + 1) * KB, E0);
            }
            compute(As + cur * KB * SA, Bs + cur * KB * SB);
            if (kt + 1 < nkt) {
                if (nedge) sstore(1 - cur, (kt + 1) * KB, E1);
                else sstore(1 - cur, (kt + 1) * KB, E0);
            }
            __syncthreads();
        }
    } else {
        if (nkt > 0) {
            if (is_edge(0)) gload(0, E1);
            else gload(0, E0);
        }
        for (int64_t kt = 0; kt < nkt; ++kt) {
            __syncthreads();
            if (is_edge(kt)) sstore(0, kt * KB, E1);
            else sstore(0, kt * KB, E0);
            __syncthreads();
            if (kt + 1 < nkt) {
                if (is_edge(kt + 1)) gload((kt + 1) * KB, E1);
                else gload((kt + 1) * KB, E0);
            }
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
                int64_t gj = j0 + wj * 64 + jb * 16 + Mfma<T>::row(lr, r);
                if (gj >= n) continue;
                T* cp = C + gi + gj * ldc;
                T v = alpha * acc[ib][jb][r];
                if (!pre && beta != T(0)) v += beta * (*cp);
                *cp = v;
            }
        }
    }
}

}  // namespace fl_tile
