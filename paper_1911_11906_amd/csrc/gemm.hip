// Dense GEMM on the CDNA4 matrix cores (tile machinery in gemm_tile.h).
//
// FP64: v_mfma_f64_16x16x4f64.  Operand layout (measured on gfx950): lane l
// supplies A[l%16][l/16] and B[l/16][l%16]; the 4 accumulator registers of
// lane l hold D[l/16 + 4r][l%16], r = 0..3.
// FP32: v_mfma_f32_16x16x4f32, same inputs, accumulator D[4(l/16) + r][l%16]
// (both through the same templated tile).
//
// We compute C^T tiles: the MFMA "A" operand is fed from op(B) and the "B"
// operand from op(A), so the 16 lanes that share an accumulator row write 16
// consecutive rows of the column-major C (128-byte segments).
//
// Workgroup tile 128 x 128, k-step 32 staged k-major in LDS with the next
// step prefetched into registers; 256 threads = 2 x 2 waves of 64 x 64.
// Problems with few output tiles and a long k are split along k into
// partial products that a second kernel sums in a fixed order.
#include <algorithm>
#include <mutex>
#include <vector>
#include "gemm_tile.h"

namespace {
using namespace fl_tile;

constexpr int GKB = 16, GNBUF = 1;  // k-step 16 with register prefetch: fits two waves per SIMD

template <class T>
struct Prob {
    int64_t m, n, k;
    const T* A;
    int64_t lda;
    const T* B;
    int64_t ldb;
    T* C;
    int64_t ldc;
    T alpha, beta;
};

// KT: zero structure of a triangular operand, used to shorten each tile's k
// range: FL_KT_A_LOWER op(A)[i][k] = 0 for k > i; FL_KT_A_UPPER for k < i;
// FL_KT_B_LOWER op(B)[k][j] = 0 for k < j.  (BM = BN is a multiple of the
// k-step, so the shortened ranges stay aligned.)
template <class T, bool TA, bool TB, bool LOWER, int KT = FL_KT_NONE, int KB = GKB>
__global__ __launch_bounds__(NT) FL_TWO_WAVES_PER_SIMD void gemm_kernel(Prob<T> g) {
    __shared__ T As[TileLds<KB, GNBUF>::A];
    __shared__ T Bs[TileLds<KB, GNBUF>::B];
    int64_t bi = blockIdx.x, bj = blockIdx.y;
    if (KT == FL_KT_A_LOWER || KT == FL_KT_A_UPPER) {
        // tiles differ in k length by row block: hand out the row blocks in
        // order of decreasing length (column blocks fastest), so the last
        // tiles to start are the short ones
        const int64_t tm = gridDim.x, tn = gridDim.y;
        const int64_t id = (int64_t)blockIdx.x + tm * blockIdx.y;
        const int64_t q = id / tn;
        bj = id - q * tn;
        bi = (KT == FL_KT_A_LOWER) ? tm - 1 - q : q;
    }
    if (LOWER && (bi + 1) * BM <= bj * BN) return;  // tile strictly above the diagonal
    int64_t kb = 0, ke = g.k;
    if (KT == FL_KT_A_LOWER) ke = std::min<int64_t>(g.k, (bi + 1) * BM);
    if (KT == FL_KT_A_UPPER) kb = std::min<int64_t>(g.k, bi * BM);
    if (KT == FL_KT_B_LOWER) kb = std::min<int64_t>(g.k, bj * BN);
    const T* A = TA ? g.A + kb : g.A + kb * g.lda;
    const T* B = TB ? g.B + kb * g.ldb : g.B + kb;
    BPlainT<T> bsrc{B, g.ldb, TB};
    tile_gemm<TA, !TB, BPlainT<T>, KB, GNBUF, T>(g.m, g.n, ke - kb, A, g.lda, bsrc, g.alpha, g.beta, g.C, g.ldc, bi,
                                                 bj, As, Bs);
}

// Lower triangle of a square tile grid: one block per tile on or below the
// diagonal (a full grid whose upper blocks exit at once ran ~25 % slower),
// tiles numbered row by row (bi slow, bj = 0..bi fast).  With KT_A_LOWER the
// k range grows with bi, so the rows are handed out last to first.
template <class T, bool TA, bool TB, int KT = FL_KT_NONE>
__global__ __launch_bounds__(NT) FL_TWO_WAVES_PER_SIMD void gemm_lower_kernel(Prob<T> g, int64_t ntiles) {
    __shared__ T As[TileLds<GKB, GNBUF>::A];
    __shared__ T Bs[TileLds<GKB, GNBUF>::B];
    const int64_t id = (KT == FL_KT_A_LOWER) ? ntiles - 1 - (int64_t)blockIdx.x : (int64_t)blockIdx.x;
    int64_t bi = (int64_t)((sqrt(8.0 * (double)id + 1.0) - 1.0) * 0.5);
    while (bi * (bi + 1) / 2 > id) --bi;
    while ((bi + 1) * (bi + 2) / 2 <= id) ++bi;
    const int64_t bj = id - bi * (bi + 1) / 2;
    int64_t kb = 0, ke = g.k;
    if (KT == FL_KT_A_LOWER) ke = std::min<int64_t>(g.k, (bi + 1) * BM);
    if (KT == FL_KT_A_UPPER) kb = std::min<int64_t>(g.k, bi * BM);
    if (KT == FL_KT_B_LOWER) kb = std::min<int64_t>(g.k, bj * BN);
    const T* A = TA ? g.A + kb : g.A + kb * g.lda;
    const T* B = TB ? g.B + kb * g.ldb : g.B + kb;
    BPlainT<T> bsrc{B, g.ldb, TB};
    tile_gemm<TA, !TB, BPlainT<T>, GKB, GNBUF, T>(g.m, g.n, ke - kb, A, g.lda, bsrc, g.alpha, g.beta, g.C, g.ldc, bi,
                                                  bj, As, Bs);
}

// Products with at most 64 columns: 256 x 64 tiles (four waves along M), so
// no half of each tile multiplies padding.  Split along k when the tiles are
// too few to fill the chip.  (One wave per SIMD: the transposed variants
// would spill at two.)
constexpr int TKB = 16, TWM = 4, TBM = 64 * TWM, TBN = 64;
template <class T, bool TA, bool TB>
__global__ __launch_bounds__(NT) void gemm_thin_kernel(Prob<T> g, int64_t kc, T* P) {
    __shared__ T As[TileLds<TKB, 1, TWM>::A];
    __shared__ T Bs[TileLds<TKB, 1, TWM>::B];
    const int64_t z = blockIdx.z;
    const int64_t koff = z * kc;
    const int64_t ks = (g.k - koff) < kc ? (g.k - koff) : kc;
    const T* A = TA ? g.A + koff : g.A + koff * g.lda;
    const T* B = TB ? g.B + koff * g.ldb : g.B + koff;
    BPlainT<T> bsrc{B, g.ldb, TB};
    // P: partial product of slice z (beta = 0) into the split-K workspace; else C directly
    const bool split = P != nullptr;
    tile_gemm<TA, !TB, BPlainT<T>, TKB, 1, T, TWM>(g.m, g.n, split ? (ks > 0 ? ks : 0) : g.k, A, g.lda, bsrc, g.alpha,
                                                   split ? T(0) : g.beta, split ? P + z * g.m * g.n : g.C,
                                                   split ? g.m : g.ldc, blockIdx.x, 0, As, Bs);
}

// Split-K: slice z of the k range into its own partial product P_z (beta = 0).
template <class T, bool TA, bool TB>
__global__ __launch_bounds__(NT) FL_TWO_WAVES_PER_SIMD void gemm_splitk_kernel(Prob<T> g, int64_t kc, T* P) {
    __shared__ T As[TileLds<GKB, GNBUF>::A];
    __shared__ T Bs[TileLds<GKB, GNBUF>::B];
    const int64_t z = blockIdx.z;
    const int64_t koff = z * kc;
    const int64_t ks = (g.k - koff) < kc ? (g.k - koff) : kc;
    const T* A = TA ? g.A + koff : g.A + koff * g.lda;
    const T* B = TB ? g.B + koff * g.ldb : g.B + koff;
    BPlainT<T> bsrc{B, g.ldb, TB};
    tile_gemm<TA, !TB, BPlainT<T>, GKB, GNBUF, T>(g.m, g.n, ks > 0 ? ks : 0, A, g.lda, bsrc, g.alpha, T(0),
                                                  P + z * g.m * g.n, g.m, blockIdx.x, blockIdx.y, As, Bs);
}

// C = beta C + sum_z P_z, fixed summation order (deterministic)
template <class T>
__global__ void splitk_reduce_kernel(int64_t m, int64_t n, int S, const T* __restrict__ P, T beta, T* C,
                                     int64_t ldc) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
        T acc = T(0);
#pragma unroll 8
        for (int z = 0; z < S; ++z) acc += P[(int64_t)z * m * n + i + j * m];
        T* c = C + i + j * ldc;
        *c = (beta != T(0)) ? beta * (*c) + acc : acc;
    }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(NT) FL_TWO_WAVES_PER_SIMD void dgemm_batched_kernel(const GemmProblem* __restrict__ probs) {
    __shared__ double As[TileLds<GKB, GNBUF>::A];
    __shared__ double Bs[TileLds<GKB, GNBUF>::B];
    const GemmProblem g = probs[blockIdx.z];
    const int64_t bi = blockIdx.x, bj = blockIdx.y;
    if (bi * BM >= g.m || bj * BN >= g.n) return;
    BPlain bsrc{g.B, g.ldb, TB};
    tile_gemm<TA, !TB, BPlain, GKB, GNBUF>(g.m, g.n, g.k, g.A, g.lda, bsrc, g.alpha, g.beta, g.C, g.ldc, bi, bj, As,
                                           Bs);
}

// Split-K workspace: one buffer per (device, stream), allocated on the
// first split product queued on that stream and kept until the process ends
// (a resize could free memory that queued kernels still use).  Products on
// different streams therefore never share partial sums; products on one
// stream are ordered by the stream.  The split factor is capped to what
// fits.
constexpr size_t SPLITK_WS_BYTES = size_t(256) << 20;
struct StreamWs {
    int dev;
    hipStream_t s;
    void* p;
};
std::mutex g_ws_mu;
std::vector<StreamWs> g_ws;
SplitWs stream_splitk_ws(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SplitWs{nullptr, 0};
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (const StreamWs& w : g_ws)
        if (w.dev == dev && w.s == s) return SplitWs{w.p, w.p ? SPLITK_WS_BYTES : 0};
    // never allocate while the stream is being captured into a graph
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s && hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return SplitWs{nullptr, 0};
    void* p = nullptr;
    if (hipMalloc(&p, SPLITK_WS_BYTES) != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
    }
    g_ws.push_back(StreamWs{dev, s, p});
    return SplitWs{p, p ? SPLITK_WS_BYTES : 0};
}

// Workspace of a split product: the caller's (ws != null; bytes == 0 means
// no split) or the stream's own buffer.
template <class T>
T* split_buffer(hipStream_t s, const SplitWs* ws, int64_t& S, int64_t m, int64_t n) {
    if (S <= 1) return nullptr;
    SplitWs w = ws ? *ws : stream_splitk_ws(s);
    while (S > 1 && (size_t)(S * m * n) * sizeof(T) > w.bytes) --S;
    if (S <= 1 || !w.p) {
        S = 1;
        return nullptr;
    }
    return static_cast<T*>(w.p);
}

template <class T, bool TA, bool TB>
hipError_t launch_thin(hipStream_t s, const Prob<T>& g, int64_t tmt, int64_t S, T* P) {
    if (S > 1 && P) {
        int64_t kc = FL_DIV_UP(FL_DIV_UP(g.k, S), TKB) * TKB;
        S = FL_DIV_UP(g.k, kc);
        gemm_thin_kernel<T, TA, TB><<<dim3((unsigned)tmt, 1, (unsigned)S), NT, 0, s>>>(g, kc, P);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        dim3 rg((unsigned)FL_DIV_UP(g.m, 256), (unsigned)std::min<int64_t>(g.n, 65535));
        splitk_reduce_kernel<T><<<rg, 256, 0, s>>>(g.m, g.n, (int)S, P, g.beta, g.C, g.ldc);
        return hipGetLastError();
    }
    gemm_thin_kernel<T, TA, TB><<<dim3((unsigned)tmt, 1, 1), NT, 0, s>>>(g, g.k, nullptr);
    return hipGetLastError();
}

// 128 x 128 tiles with k-step kb (16 or 32), optionally split along k.
template <class T, bool TA, bool TB>
hipError_t launch_square(hipStream_t s, const Prob<T>& g, int kb, int64_t S, T* P) {
    const int64_t tm = FL_DIV_UP(g.m, BM), tn = FL_DIV_UP(g.n, BN);
    if (S > 1 && P) {
        int64_t kc = FL_DIV_UP(FL_DIV_UP(g.k, S), GKB) * GKB;
        S = FL_DIV_UP(g.k, kc);
        gemm_splitk_kernel<T, TA, TB><<<dim3((unsigned)tm, (unsigned)tn, (unsigned)S), NT, 0, s>>>(g, kc, P);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        dim3 rg((unsigned)FL_DIV_UP(g.m, 256), (unsigned)std::min<int64_t>(g.n, 65535));
        splitk_reduce_kernel<T><<<rg, 256, 0, s>>>(g.m, g.n, (int)S, P, g.beta, g.C, g.ldc);
        return hipGetLastError();
    }
    dim3 grid((unsigned)tm, (unsigned)tn);
    if (kb == 2 * GKB)
        gemm_kernel<T, TA, TB, false, FL_KT_NONE, 2 * GKB><<<grid, NT, 0, s>>>(g);
    else
        gemm_kernel<T, TA, TB, false><<<grid, NT, 0, s>>>(g);
    return hipGetLastError();
}

template <class T, bool TA, bool TB>
hipError_t launch(hipStream_t s, const Prob<T>& g, int lower, const SplitWs* ws, const GemmChoice* forced) {
    const GemmChoice tc = forced ? *forced
                                 : lower ? GemmChoice{}
                                         : tuned_choice(sizeof(T) == 8 ? FL_TUNE_F64 : FL_TUNE_F32, TA, TB, g.m, g.n,
                                                        g.k);
    if (tc.variant == FL_GV_THIN && g.n <= TBN) {
        const int64_t tmt = FL_DIV_UP(g.m, TBM);
        int64_t S = std::max<int64_t>(1, std::min<int64_t>(tc.split, g.k / TKB));
        T* P = split_buffer<T>(s, ws, S, g.m, g.n);
        return launch_thin<T, TA, TB>(s, g, tmt, S, P);
    }
    if (tc.variant == FL_GV_SQUARE16 || tc.variant == FL_GV_SQUARE32) {
        const int kb = tc.variant == FL_GV_SQUARE32 ? 2 * GKB : GKB;
        int64_t S = std::max<int64_t>(1, std::min<int64_t>(tc.split, g.k / kb));
        T* P = split_buffer<T>(s, ws, S, g.m, g.n);
        return launch_square<T, TA, TB>(s, g, kb, S, P);
    }
    if (!lower && g.n <= TBN && g.m >= 2 * TBM) {
        const int64_t tmt = FL_DIV_UP(g.m, TBM);
        int64_t S = 1;
        T* P = nullptr;
        if (tmt < 384 && g.k >= 256) {
            S = std::min<int64_t>({FL_DIV_UP(768, tmt), g.k / 128, 32});
            P = split_buffer<T>(s, ws, S, g.m, g.n);
        }
        if (S > 1) {
            int64_t kc = FL_DIV_UP(FL_DIV_UP(g.k, S), TKB) * TKB;
            S = FL_DIV_UP(g.k, kc);
            gemm_thin_kernel<T, TA, TB><<<dim3((unsigned)tmt, 1, (unsigned)S), NT, 0, s>>>(g, kc, P);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            dim3 rg((unsigned)FL_DIV_UP(g.m, 256), (unsigned)std::min<int64_t>(g.n, 65535));
            splitk_reduce_kernel<T><<<rg, 256, 0, s>>>(g.m, g.n, (int)S, P, g.beta, g.C, g.ldc);
            return hipGetLastError();
        }
        gemm_thin_kernel<T, TA, TB><<<dim3((unsigned)tmt, 1, 1), NT, 0, s>>>(g, g.k, nullptr);
        return hipGetLastError();
    }
    const int64_t tm = FL_DIV_UP(g.m, BM), tn = FL_DIV_UP(g.n, BN);
    const int64_t tiles = tm * tn;
    // few output tiles and a long k: split k so that the chip fills up (down
    // to k-slices of 128 for the smallest outputs, e.g. the 64 x 64 Gram
    // matrices of the band reduction); a handful of tiles with a moderate k
    // (the block steps of the banded Cholesky: one or two 128 x 128 tiles,
    // k = 128 .. 512) in slices of 32 (a single tile may be a lower one: the
    // lower kernel writes whole diagonal tiles as well)
    const bool few = (!lower || tiles == 1) && tiles <= 16 && g.k >= 128 && g.k < 1024;
    if ((!lower && tiles < 384 && g.k >= 1024) || few) {
        int64_t S = few ? std::min<int64_t>(g.k / 32, FL_DIV_UP(512, tiles))
                        : std::min<int64_t>({FL_DIV_UP(1024, tiles), g.k / 128, 256});
        T* P = split_buffer<T>(s, ws, S, g.m, g.n);
        if (S > 1 && P) {
            int64_t kc = FL_DIV_UP(FL_DIV_UP(g.k, S), GKB) * GKB;
            S = FL_DIV_UP(g.k, kc);
            gemm_splitk_kernel<T, TA, TB><<<dim3((unsigned)tm, (unsigned)tn, (unsigned)S), NT, 0, s>>>(g, kc, P);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            dim3 rg((unsigned)FL_DIV_UP(g.m, 256), (unsigned)std::min<int64_t>(g.n, 65535));
            splitk_reduce_kernel<T><<<rg, 256, 0, s>>>(g.m, g.n, (int)S, P, g.beta, g.C, g.ldc);
            return hipGetLastError();
        }
    }
    dim3 grid((unsigned)tm, (unsigned)tn);
    // long FP32 products: k-step 32 fits the same registers and LDS bytes as
    // FP64's 16 and halves the barriers per flop
    if (!lower && sizeof(T) == 4 && g.k >= 8192) {
        gemm_kernel<T, TA, TB, false, FL_KT_NONE, 2 * GKB><<<grid, NT, 0, s>>>(g);
        return hipGetLastError();
    }
    if (lower && tm == tn) {
        const int64_t nt = tm * (tm + 1) / 2;
        gemm_lower_kernel<T, TA, TB><<<(unsigned)nt, NT, 0, s>>>(g, nt);
    } else if (lower)
        gemm_kernel<T, TA, TB, true><<<grid, NT, 0, s>>>(g);
    else
        gemm_kernel<T, TA, TB, false><<<grid, NT, 0, s>>>(g);
    return hipGetLastError();
}

template <int KT, bool TA, bool TB>
hipError_t launch_tri(hipStream_t s, const Prob<double>& g, int lower) {
    dim3 grid((unsigned)FL_DIV_UP(g.m, BM), (unsigned)FL_DIV_UP(g.n, BN));
    if (lower && grid.x == grid.y) {
        const int64_t nt = (int64_t)grid.x * (grid.x + 1) / 2;
        gemm_lower_kernel<double, TA, TB, KT><<<(unsigned)nt, NT, 0, s>>>(g, nt);
    } else if (lower)
        gemm_kernel<double, TA, TB, true, KT><<<grid, NT, 0, s>>>(g);
    else
        gemm_kernel<double, TA, TB, false, KT><<<grid, NT, 0, s>>>(g);
    return hipGetLastError();
}

template <int KT>
hipError_t tri_any(hipStream_t s, int ta, int tb, const Prob<double>& g, int lower) {
    if (!ta && !tb) return launch_tri<KT, false, false>(s, g, lower);
    if (!ta && tb) return launch_tri<KT, false, true>(s, g, lower);
    if (ta && !tb) return launch_tri<KT, true, false>(s, g, lower);
    return launch_tri<KT, true, true>(s, g, lower);
}

template <class T>
hipError_t gemm_any(hipStream_t s, int ta, int tb, const Prob<T>& g, int lower, const SplitWs* ws = nullptr,
                    const GemmChoice* forced = nullptr) {
    if (!ta && !tb) return launch<T, false, false>(s, g, lower, ws, forced);
    if (!ta && tb) return launch<T, false, true>(s, g, lower, ws, forced);
    if (ta && !tb) return launch<T, true, false>(s, g, lower, ws, forced);
    return launch<T, true, true>(s, g, lower, ws, forced);
}

// ---------------------------------------------------------------- helpers
template <class S, class D>
__global__ void convert_kernel(int64_t m, int64_t n, const S* __restrict__ A, int64_t lda, D* __restrict__ B,
                               int64_t ldb) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        if (i < m) B[i + j * ldb] = (D)A[i + j * lda];
}

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

// A(i, j) = A(j, i) for i < j (upper from lower), 32 x 32 tiles through LDS.
template <class T>
__global__ void mirror_lower_kernel(int64_t n, T* A, int64_t lda) {
    __shared__ T tile[32][33];
    const int64_t bi = blockIdx.x, bj = blockIdx.y;  // source tile (bi, bj) with bi >= bj
    if (bi < bj) return;
    const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = bi * 32 + tx, j = bj * 32 + r;
        if (i < n && j < n) tile[r][tx] = A[i + j * lda];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = bj * 32 + tx, j = bi * 32 + r;  // destination (i, j) = source (j, i)
        if (i < n && j < n && i < j) A[i + j * lda] = tile[tx][r];
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
    Prob<double> g{m, n, k, A, lda, B, ldb, C, ldc, alpha, beta};
    return gemm_any<double>(s, ta, tb, g, lower);
}

SplitWs fl_stream_splitk_ws(hipStream_t s) { return stream_splitk_ws(s); }

hipError_t fl_dgemm_ws(hipStream_t s, int ta, int tb, int64_t m, int64_t n, int64_t k, double alpha,
                       const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                       int64_t ldc, const SplitWs* ws) {
    if (m <= 0 || n <= 0) return hipSuccess;
    if (k <= 0 && beta == 1.0) return hipSuccess;
    Prob<double> g{m, n, k, A, lda, B, ldb, C, ldc, alpha, beta};
    SplitWs none{nullptr, 0};
    return gemm_any<double>(s, ta, tb, g, 0, ws ? ws : &none);
}

hipError_t fl_gemm_choice_launch(hipStream_t s, int dtype, int ta, int tb, int64_t m, int64_t n, int64_t k,
                                 const void* A, int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc,
                                 const GemmChoice& c) {
    if (m <= 0 || n <= 0 || k <= 0) return hipSuccess;
    if (dtype == FL_TUNE_F32) {
        Prob<float> g{m, n, k, (const float*)A, lda, (const float*)B, ldb, (float*)C, ldc, 1.0f, 0.0f};
        return gemm_any<float>(s, ta, tb, g, 0, nullptr, &c);
    }
    Prob<double> g{m, n, k, (const double*)A, lda, (const double*)B, ldb, (double*)C, ldc, 1.0, 0.0};
    return gemm_any<double>(s, ta, tb, g, 0, nullptr, &c);
}

hipError_t fl_dgemm_tri(hipStream_t s, int ta, int tb, int64_t m, int64_t n, int64_t k, double alpha,
                        const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                        int64_t ldc, int lower, int kt) {
    if (m <= 0 || n <= 0) return hipSuccess;
    if (k <= 0 && beta == 1.0) return hipSuccess;
    Prob<double> g{m, n, k, A, lda, B, ldb, C, ldc, alpha, beta};
    switch (kt) {
        case FL_KT_A_LOWER: return tri_any<FL_KT_A_LOWER>(s, ta, tb, g, lower);
        case FL_KT_A_UPPER: return tri_any<FL_KT_A_UPPER>(s, ta, tb, g, lower);
        case FL_KT_B_LOWER: return tri_any<FL_KT_B_LOWER>(s, ta, tb, g, lower);
        default: return gemm_any<double>(s, ta, tb, g, lower);
    }
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
                    int64_t lda, const float* B, int64_t ldb, float beta, float* C, int64_t ldc, int lower) {
    if (m <= 0 || n <= 0) return hipSuccess;
    if (k <= 0 && beta == 1.0f) return hipSuccess;
    Prob<float> g{m, n, k, A, lda, B, ldb, C, ldc, alpha, beta};
    return gemm_any<float>(s, ta, tb, g, lower);
}

hipError_t fl_d2s(hipStream_t s, int64_t m, int64_t n, const double* A, int64_t lda, float* B, int64_t ldb) {
    if (m <= 0 || n <= 0) return hipSuccess;
    convert_kernel<double, float><<<grid2(m, n), 256, 0, s>>>(m, n, A, lda, B, ldb);
    return hipGetLastError();
}

hipError_t fl_s2d(hipStream_t s, int64_t m, int64_t n, const float* A, int64_t lda, double* B, int64_t ldb) {
    if (m <= 0 || n <= 0) return hipSuccess;
    convert_kernel<float, double><<<grid2(m, n), 256, 0, s>>>(m, n, A, lda, B, ldb);
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

hipError_t fl_mirror_lower(hipStream_t s, int64_t n, double* A, int64_t lda) {
    if (n <= 1) return hipSuccess;
    dim3 grid((unsigned)FL_DIV_UP(n, 32), (unsigned)FL_DIV_UP(n, 32));
    mirror_lower_kernel<double><<<grid, dim3(32, 8), 0, s>>>(n, A, lda);
    return hipGetLastError();
}
hipError_t fl_mirror_lower_f(hipStream_t s, int64_t n, float* A, int64_t lda) {
    if (n <= 1) return hipSuccess;
    dim3 grid((unsigned)FL_DIV_UP(n, 32), (unsigned)FL_DIV_UP(n, 32));
    mirror_lower_kernel<float><<<grid, dim3(32, 8), 0, s>>>(n, A, lda);
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
