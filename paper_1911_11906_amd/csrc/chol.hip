// Cholesky of the mass matrix (M = L L^T) and the triangular solves that
// bring the pencil to standard form (C = L^-1 K L^-T) and map eigenvectors
// back (V = L^-T Z), all in FP64.
//
// Recursive blocking on 128-aligned splits: every leaf is a 128 x 128
// diagonal block, factored by one workgroup (the block in registers) that
// also inverts it.  Off-diagonal work is GEMM (matrix cores); a triangular
// solve at a leaf is a GEMM with the stored leaf inverse.  A banded M keeps
// its band: left-looking block steps over the band, and solves with many
// right-hand sides as one strip-parallel launch (the end of this file).
#include <algorithm>
#include "internal.h"

namespace {

constexpr int LB = 128;  // leaf block
constexpr int LT = 1024; // threads of the leaf kernel

// v moved across the lanes of a wave by the DPP control CTRL (both halves)
template <int CTRL>
__device__ inline double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the eight aligned lanes 8r .. 8r+7: swaps within pairs and within
// quads, then the mirror within each half row of eight lanes; every lane of
// the eight gets the same bits (each step adds a and b in either order).
__device__ inline double sum8(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    return v;
}

// Inverse X of the lower-triangular LB x LB block L in LDS (column-major, ld
// LB), written to out (LB x LB, zero above the diagonal).  X L = I gives, row
// by row from the right, X_ii = 1 / L_ii and
//     X_ij = -(1 / L_jj) sum_{k = j+1..i} X_ik L_kj   (j < i),
// which uses only row i of X: eight lanes own row i (lane p keeps X_ik for
// k = p mod 8 in registers) and split each sum, so no workgroup barrier is
// needed.  L is only read.
// rdiag: 1 / L_jj (LB entries).  The sums run over every k without a
// condition: at step j the registers hold X_ik only for k in (j, i] and zero
// elsewhere (entries are set at step k = j only for j <= i), so the other
// products vanish, and the LDS reads of a step issue back to back.
__device__ void invert_lower_rows(const double* L, const double* rdiag, double* out, int t) {
    const int i = t >> 3, part = t & 7;  // 1024 threads: 128 rows x 8 lanes
    double X[LB / 8];
#pragma unroll
    for (int q = 0; q < LB / 8; ++q) X[q] = 0.0;
    for (int j = LB - 1; j >= 0; --j) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < LB / 8; ++q) {
            acc += X[q] * L[8 * q + part + j * LB];
        }
        acc = sum8(acc);
        const double x = (j == i) ? rdiag[j] : -acc * rdiag[j];
        if (j <= i && part == (j & 7)) {
#pragma unroll
            for (int q = 0; q < LB / 8; ++q)
                if (q == (j >> 3)) X[q] = x;
        }
    }
#pragma unroll
    for (int q = 0; q < LB / 8; ++q) {
        const int k = 8 * q + part;
        out[i + k * LB] = (k <= i) ? X[q] : 0.0;
    }
}

// Factor the nb x nb (nb <= 128) diagonal block at A (ld lda); write L back
// (strict upper triangle of the block zeroed) and its inverse (128 x 128,
// zero padded) to Linv.  info: first failing global pivot (1-based) if unset.
// 256 threads; thread t holds the 8 x 8 register block (rows 8 (t mod 16)..,
// columns 8 (t / 16)..), so a step reads 16 values from LDS per thread
// (32 KB per step for the workgroup, where one value per entry held would
// read 128 KB) for 64 multiply-adds.  Step j: the owners of column j publish
// it in LDS (two buffers by parity, one barrier per step) and every block
// with columns c > j updates S_ic -= S_ij S_cj / d_j, keeping the columns
// unscaled; L = column c / sqrt(d_c) is formed at the end.  A pivot d_j <= 0
// is reported and replaced by 1 (every thread derives the same replacement
// from the value it reads).  Padding rows and columns (>= nb) are the
// identity, which keeps the inverse well defined.  The inverse solves
// L X = I by rows in the same layout: row i of X is final once rows < i are
// (X_i = (e_i - sum_{k<i} L_ik X_k) / L_ii); it is published and every block
// below subtracts L_mi X_i from its rows m > i.
constexpr int LT2 = 256;  // threads of the leaf kernel
__global__ __launch_bounds__(LT2) void potrf_leaf_kernel(double* A, int64_t lda, int nb, int64_t goff,
                                                         double* Linv, int64_t* info) {
    __shared__ __attribute__((aligned(16))) double S[LB * LB];  // L, column-major with ld LB
    __shared__ __attribute__((aligned(16))) double pv[2][LB];   // published column (factor) or row (inverse), by parity
    __shared__ double dg[LB];                                   // pivots (1 for padding)
    __shared__ double rd[LB];                                   // 1 / L_jj
    const int t = threadIdx.x;
    const int br = t & 15, bc = t >> 4;  // row block, column block
    const int i0 = 8 * br, c0 = 8 * bc;
    double X[8][8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
            const int i = i0 + r, c = c0 + cc;
            X[r][cc] = (i < nb && c < nb) ? ((i >= c) ? A[i + (int64_t)c * lda] : 0.0) : ((i == c) ? 1.0 : 0.0);
        }
    if (t < LB) dg[t] = 1.0;
    bool bad = false;  // thread 0 only
    // 8 consecutive doubles of pv starting at a multiple of 8
    auto read8 = [&](const double* p, double (&v)[8]) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const double2 w = *reinterpret_cast<const double2*>(p + 2 * h);
            v[2 * h] = w.x;
            v[2 * h + 1] = w.y;
        }
    };
    for (int jb = 0; jb < LB / 8; ++jb) {
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const int j = 8 * jb + jj;
            if (j >= nb) break;  // uniform
            double* cj = pv[j & 1];
            if (bc == jb) {
#pragma unroll
                for (int r = 0; r < 8; ++r) cj[i0 + r] = X[r][jj];
            }
            __syncthreads();
            const double d = cj[j];
            const double deff = (d > 0.0) ? d : 1.0;
            if (t == 0) {
                if (!(d > 0.0) && !bad && *info == 0) *info = goff + j + 1;
                bad = bad || !(d > 0.0);
                dg[j] = deff;
            }
            // blocks left of or at column j (except j's own later columns) are finished
            if (bc >= jb && br >= bc) {
                double prow[8], pcol[8];
                read8(cj + i0, prow);
                read8(cj + c0, pcol);
                const double rinv = 1.0 / deff;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const double sij = prow[r] * rinv;
#pragma unroll
                    for (int cc = 0; cc < 8; ++cc)
                        if (bc > jb || cc > jj) X[r][cc] = fma(-sij, pcol[cc], X[r][cc]);
                }
            }
        }
    }
    __syncthreads();
    if (t < LB) {
        const double y = sqrt(dg[t]);
        pv[0][t] = y;
        rd[t] = 1.0 / y;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
            const int i = i0 + r, c = c0 + cc;
            const double v = (i > c) ? X[r][cc] / pv[0][c] : ((i == c) ? pv[0][c] : 0.0);
            S[i + c * LB] = v;
            if (i < nb && c < nb) A[i + (int64_t)c * lda] = v;
            X[r][cc] = (i == c) ? 1.0 : 0.0;  // the inverse's right-hand side I
        }
    __syncthreads();
    // rows of X = L^-1, ascending; X holds the partial right-hand sides
    for (int ib = 0; ib < LB / 8; ++ib) {
#pragma unroll
        for (int ii = 0; ii < 8; ++ii) {
            const int i = 8 * ib + ii;
            double* xi = pv[i & 1];
            if (br == ib) {
                const double s = rd[i];
#pragma unroll
                for (int cc = 0; cc < 8; ++cc) {
                    X[ii][cc] *= s;
                    xi[c0 + cc] = X[ii][cc];
                }
            }
            __syncthreads();
            // rows m > i of blocks on or below the diagonal: X_m -= L_mi X_i
            if (br >= ib && br >= bc && c0 <= i) {
                double lcol[8], xrow[8];
                read8(S + i * LB + i0, lcol);
                read8(xi + c0, xrow);
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    if (br > ib || r > ii) {
#pragma unroll
                        for (int cc = 0; cc < 8; ++cc) X[r][cc] = fma(-lcol[r], xrow[cc], X[r][cc]);
                    }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
            const int i = i0 + r, c = c0 + cc;
            Linv[i + c * LB] = (c <= i) ? X[r][cc] : 0.0;
        }
}

// Inverses of the 128 x 128 diagonal blocks of an existing lower factor L
// (one workgroup per block).
__global__ __launch_bounds__(LT) void trtri_leaves_kernel(int64_t n, const double* L, int64_t ldl, double* Linv) {
    __shared__ double S[LB * LB];
    __shared__ double rd[LB];
    const int t = threadIdx.x;
    const int64_t off = (int64_t)blockIdx.x * LB;
    const int nb = (int)((n - off) < LB ? (n - off) : LB);
    for (int e = t; e < LB * LB; e += LT) {
        int i = e % LB, j = e / LB;
        S[i + j * LB] = (i < nb && j < nb) ? ((i >= j) ? L[off + i + (off + j) * ldl] : 0.0) : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    if (t < LB) rd[t] = 1.0 / S[t + t * LB];
    __syncthreads();
    invert_lower_rows(S, rd, Linv + (int64_t)blockIdx.x * LB * LB, t);
}

__global__ void symmetrize_kernel(int64_t n, double* A, int64_t lda) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t j = blockIdx.y;
    for (; j < n; j += gridDim.y) {
        if (i < n && i > j) {
            double v = 0.5 * (A[i + j * lda] + A[j + i * lda]);
            A[i + j * lda] = v;
            A[j + i * lda] = v;
        }
    }
}

inline int64_t split_point(int64_t k) {
    int64_t leaves = FL_DIV_UP(k, LB);
    return LB * ((leaves + 1) / 2);
}


// ------------------------------------------- banded solves, column strips
// For many right-hand sides the banded substitution runs as one launch: each
// workgroup owns a strip of BSW columns of B and walks all block rows in
// turn, so no workgroup ever waits for another.  Block row i becomes one
// product X_i = P_i B[lo_i : lo_i + K_i, strip] with a precomputed panel
//   forward  (L X = B):   P_i = [ -L_ii^-1 L_i,k  |  L_ii^-1 ],  lo_i = k0
//   backward (L^T X = B): P_i = [ L_ii^-T  |  -L_ii^-T L_k,i^T ], lo_i = i0
// (k the q block rows on the far side of the diagonal block), which reads
// the already solved rows and B_i together; X_i overwrites B_i once every
// wave has read it.
constexpr int BSW = 64;  // strip width
constexpr int BSK = 32;  // k-slab staged in LDS

__device__ inline void band_row_range(bool back, int64_t n, int64_t q, int64_t i, int64_t& i0, int64_t& nb,
                                      int64_t& lo, int64_t& K) {
    i0 = i * LB;
    nb = (n - i0) < LB ? (n - i0) : LB;
    if (!back) {
        lo = (i > q ? i - q : 0) * LB;
        K = i0 + nb - lo;
    } else {
        lo = i0;
        const int64_t r1 = i0 + nb, w = (n - r1) < q * LB ? (n - r1) : q * LB;
        K = nb + w;
    }
}

// Diagonal parts of the panels: L_ii^-1 (forward, after the w = i0 - k0
// columns of the off-diagonal part) or L_ii^-T (backward, first).  One
// workgroup per block row.
template <bool BACK>
__global__ void band_panel_diag_kernel(int64_t n, int64_t q, const double* __restrict__ Linv, double* P) {
    const int64_t i = blockIdx.x, KP = (q + 1) * LB;
    int64_t i0, nb, lo, K;
    band_row_range(BACK, n, q, i, i0, nb, lo, K);
    const double* Li = Linv + i * LB * LB;
    double* Pi = P + i * LB * KP;
    const int64_t off = BACK ? 0 : i0 - lo;
    for (int e = threadIdx.x; e < LB * LB; e += blockDim.x) {
        const int r = e % LB, c = e / LB;
        Pi[r + (off + c) * LB] = BACK ? Li[c + r * LB] : Li[r + c * LB];
    }
}

// acc row/column of lane (lr, lc), register r: row 16 ti + lc of the wave's
// 32 rows, column 16 tj + lr + 4 r (the MFMA's first operand is fed from B).
template <bool BACK>
__global__ __launch_bounds__(256) void band_solve_kernel(int64_t n, int64_t q, const double* __restrict__ P,
                                                         double* B, int64_t ldb, int64_t ncols, int64_t bwb) {
    __shared__ double As[BSK][LB + 2];   // As[k][r] = P_i(r, kk + k)
    __shared__ double Bs[BSK][BSW + 2];  // Bs[k][j] = B(lo + kk + k, c0 + j)
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int lr = lane >> 4, lc = lane & 15;
    const int64_t c0 = (int64_t)blockIdx.x * BSW;
    const int64_t nbk = FL_DIV_UP(n, LB), KP = (q + 1) * LB;
    constexpr int NA = BSK * LB / 256, NB = BSK * BSW / 256;  // staged elements per thread
    for (int64_t st = 0; st < nbk; ++st) {
        const int64_t i = BACK ? nbk - 1 - st : st;
        int64_t i0, nb, lo, K;
        band_row_range(BACK, n, q, i, i0, nb, lo, K);
        // forward with a banded B: rows r of B and X are zero beyond column
        // r + bwb, so a block row ending before the strip stays zero
        if (!BACK && bwb >= 0 && i0 + nb - 1 + bwb < c0) continue;
        const double* Pi = P + i * LB * KP;
        d4_t acc[2][4];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] = d4_t{0, 0, 0, 0};
        double ra[NA], rb[NB];
        // slab kk into registers: loads from clamped indices, masked when staged
        auto gload = [&](int64_t kk) {
#pragma unroll
            for (int u = 0; u < NA; ++u) {
                const int e = t + 256 * u, r = e % LB, k = e / LB;
                const int64_t kc = (kk + k < K) ? kk + k : K - 1;
                ra[u] = Pi[r + kc * LB];
            }
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int e = t + 256 * u, k = e % BSK, j = e / BSK;
                const int64_t row = lo + ((kk + k < K) ? kk + k : K - 1);
                const int64_t col = (c0 + j < ncols) ? c0 + j : ncols - 1;
                rb[u] = B[row + col * ldb];
            }
        };
        gload(0);
        for (int64_t kk = 0; kk < K; kk += BSK) {
            __syncthreads();  // the previous slab has been consumed
#pragma unroll
            for (int u = 0; u < NA; ++u) {
                const int e = t + 256 * u, r = e % LB, k = e / LB;
                As[k][r] = (kk + k < K && r < nb) ? ra[u] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int e = t + 256 * u, k = e % BSK, j = e / BSK;
                Bs[k][j] = (kk + k < K) ? rb[u] : 0.0;
            }
            __syncthreads();
            if (kk + BSK < K) gload(kk + BSK);
#pragma unroll
            for (int k4 = 0; k4 < BSK; k4 += 4) {
                double fa[4], fb[2];
#pragma unroll
                for (int y = 0; y < 4; ++y) fa[y] = Bs[k4 + lr][16 * y + lc];
#pragma unroll
                for (int x = 0; x < 2; ++x) fb[x] = As[k4 + lr][wave * 32 + 16 * x + lc];
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[y], fb[x], acc[x][y], 0, 0, 0);
            }
        }
        __syncthreads();  // every wave has read B_i (part of the operand rows)
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            const int r = wave * 32 + 16 * x + lc;
#pragma unroll
            for (int y = 0; y < 4; ++y)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t col = c0 + 16 * y + lr + 4 * v;
                    if (r < nb && col < ncols) B[i0 + r + col * ldb] = acc[x][y][v];
                }
        }
        // the next block row reads these rows through other waves: drain the
        // stores, barrier, and drop stale vector-L1 lines
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
}
}  // namespace

int64_t fl_potrf_linv_elems(int64_t n) { return FL_DIV_UP(n, LB) * LB * LB; }
int64_t fl_trsm_work_elems(int64_t n, int64_t other) { (void)n; return (int64_t)LB * (other > 0 ? other : 1); }

hipError_t fl_potrf(hipStream_t s, int64_t n, double* A, int64_t lda, double* Linv, int64_t* info, double* work) {
    if (n <= 0) return hipSuccess;
    if (n <= LB) {
        potrf_leaf_kernel<<<1, LT2, 0, s>>>(A, lda, (int)n, 0, Linv, info);
        return hipGetLastError();
    }
    // The global pivot offset of each leaf is needed in the status; recurse
    // with an explicit offset through a small lambda.
    struct Rec {
        static hipError_t run(hipStream_t s, int64_t n, double* A, int64_t lda, double* Linv, int64_t* info,
                              double* work, int64_t goff) {
            if (n <= LB) {
                potrf_leaf_kernel<<<1, LT2, 0, s>>>(A, lda, (int)n, goff, Linv, info);
                return hipGetLastError();
            }
            int64_t n1 = split_point(n), n2 = n - n1;
            hipError_t e = run(s, n1, A, lda, Linv, info, work, goff);
            if (e != hipSuccess) return e;
            e = fl_trsm_rlt(s, n2, n1, A, lda, Linv, A + n1, lda, work);
            if (e != hipSuccess) return e;
            e = fl_dgemm(s, 0, 1, n2, n2, n1, -1.0, A + n1, lda, A + n1, lda, 1.0, A + n1 + n1 * lda, lda, 1);
            if (e != hipSuccess) return e;
            return run(s, n2, A + n1 + n1 * lda, lda, Linv + (n1 / LB) * LB * LB, info, work, goff + n1);
        }
    };
    return Rec::run(s, n, A, lda, Linv, info, work, 0);
}

// X L^T = B, B is m x k.  work: >= m * 128 doubles.
hipError_t fl_trsm_rlt(hipStream_t s, int64_t m, int64_t k, const double* L, int64_t ldl, const double* Linv,
                       double* B, int64_t ldb, double* work) {
    if (m <= 0 || k <= 0) return hipSuccess;
    hipError_t e;
    if (k <= LB) {
        e = fl_copy_matrix(s, m, k, B, ldb, work, m);
        if (e != hipSuccess) return e;
        return fl_dgemm(s, 0, 1, m, k, k, 1.0, work, m, Linv, LB, 0.0, B, ldb);
    }
    int64_t k1 = split_point(k), k2 = k - k1;
    e = fl_trsm_rlt(s, m, k1, L, ldl, Linv, B, ldb, work);
    if (e != hipSuccess) return e;
    e = fl_dgemm(s, 0, 1, m, k2, k1, -1.0, B, ldb, L + k1, ldl, 1.0, B + k1 * ldb, ldb);
    if (e != hipSuccess) return e;
    return fl_trsm_rlt(s, m, k2, L + k1 + k1 * ldl, ldl, Linv + (k1 / LB) * LB * LB, B + k1 * ldb, ldb, work);
}

// L X = B, B is k x m.  work: >= 128 * m doubles.
hipError_t fl_trsm_lln(hipStream_t s, int64_t k, int64_t m, const double* L, int64_t ldl, const double* Linv,
                       double* B, int64_t ldb, double* work) {
    if (m <= 0 || k <= 0) return hipSuccess;
    hipError_t e;
    if (k <= LB) {
        e = fl_copy_matrix(s, k, m, B, ldb, work, k);
        if (e != hipSuccess) return e;
        return fl_dgemm(s, 0, 0, k, m, k, 1.0, Linv, LB, work, k, 0.0, B, ldb);
    }
    int64_t k1 = split_point(k), k2 = k - k1;
    e = fl_trsm_lln(s, k1, m, L, ldl, Linv, B, ldb, work);
    if (e != hipSuccess) return e;
    e = fl_dgemm(s, 0, 0, k2, m, k1, -1.0, L + k1, ldl, B, ldb, 1.0, B + k1, ldb);
    if (e != hipSuccess) return e;
    return fl_trsm_lln(s, k2, m, L + k1 + k1 * ldl, ldl, Linv + (k1 / LB) * LB * LB, B + k1, ldb, work);
}

// L^T X = B, B is k x m.  work: >= 128 * m doubles.
hipError_t fl_trsm_llt(hipStream_t s, int64_t k, int64_t m, const double* L, int64_t ldl, const double* Linv,
                       double* B, int64_t ldb, double* work) {
    if (m <= 0 || k <= 0) return hipSuccess;
    hipError_t e;
    if (k <= LB) {
        e = fl_copy_matrix(s, k, m, B, ldb, work, k);
        if (e != hipSuccess) return e;
        return fl_dgemm(s, 1, 0, k, m, k, 1.0, Linv, LB, work, k, 0.0, B, ldb);
    }
    int64_t k1 = split_point(k), k2 = k - k1;
    e = fl_trsm_llt(s, k2, m, L + k1 + k1 * ldl, ldl, Linv + (k1 / LB) * LB * LB, B + k1, ldb, work);
    if (e != hipSuccess) return e;
    e = fl_dgemm(s, 1, 0, k1, m, k2, -1.0, L + k1, ldl, B + k1, ldb, 1.0, B, ldb);
    if (e != hipSuccess) return e;
    return fl_trsm_llt(s, k1, m, L, ldl, Linv, B, ldb, work);
}

// In place: L (n x n lower, ld ldl) := L^-1, strict upper triangle zeroed.
// Linv: the diagonal leaves' inverses from fl_potrf.  With the same
// 128-aligned splits, [L11 0; L21 L22]^-1 = [X11 0; -X22 L21 X11  X22], the
// two products skipping the zero tiles of the triangular factors.
// work: >= n * n / 2 doubles.
hipError_t fl_trtri_inplace(hipStream_t s, int64_t n, double* L, int64_t ldl, const double* Linv, double* work) {
    if (n <= 0) return hipSuccess;
    hipError_t e;
    if (n <= LB) return fl_copy_matrix(s, n, n, Linv, LB, L, ldl);
    const int64_t n1 = split_point(n), n2 = n - n1;
    double* L22 = L + n1 + n1 * ldl;
    if ((e = fl_trtri_inplace(s, n1, L, ldl, Linv, work))) return e;
    if ((e = fl_trtri_inplace(s, n2, L22, ldl, Linv + (n1 / LB) * LB * LB, work))) return e;
    // T = L21 X11 (X11 lower), then X21 = -X22 T (X22 lower)
    if ((e = fl_dgemm_tri(s, 0, 0, n2, n1, n1, 1.0, L + n1, ldl, L, ldl, 0.0, work, n2, 0, FL_KT_B_LOWER))) return e;
    if ((e = fl_dgemm_tri(s, 0, 0, n2, n1, n2, -1.0, L22, ldl, work, n2, 0.0, L + n1, ldl, 0, FL_KT_A_LOWER))) return e;
    return fl_fill(s, n1, n2, 0.0, L + n1 * ldl, ldl);
}

// ---------------------------------------------------------------- banded M
// For a mass matrix whose half-bandwidth bw is small against n, the factor
// keeps the band (a product L_ik L_jk^T is non-zero only if both lie in the
// band), so everything runs on 128-row block rows of the band: q =
// ceil(bw / 128) blocks below each diagonal block.  The diagonal blocks are
// the same 128 x 128 leaves (factored and inverted in LDS); the rest are
// GEMMs of one block row against at most q neighbouring block rows.

// Left-looking block Cholesky restricted to the band: for each block column
// j, S = A_jj - L_j,k L_j,k^T (k in [j-q, j)), L_jj = chol(S) with its
// inverse, then the q blocks below: L_ij = (A_ij - L_i,k L_j,k^T) L_jj^-T.
// Entries outside the band must be zero on entry and stay zero.
hipError_t fl_potrf_band(hipStream_t s, int64_t n, int64_t q, double* A, int64_t lda, double* Linv, int64_t* info,
                         double* work) {
    if (n <= 0) return hipSuccess;
    const int64_t nbk = FL_DIV_UP(n, LB);
    hipError_t e;
    for (int64_t j = 0; j < nbk; ++j) {
        const int64_t j0 = j * LB, nb = std::min<int64_t>(LB, n - j0);
        const int64_t k0 = std::max<int64_t>(0, j - q) * LB, w = j0 - k0;  // columns of the left neighbours
        double* Ajj = A + j0 + j0 * lda;
        if (w > 0 && (e = fl_dgemm(s, 0, 1, nb, nb, w, -1.0, A + j0 + k0 * lda, lda, A + j0 + k0 * lda, lda, 1.0, Ajj,
                                   lda, 1)))
            return e;
        potrf_leaf_kernel<<<1, LT2, 0, s>>>(Ajj, lda, (int)nb, j0, Linv + j * LB * LB, info);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int64_t r1 = j0 + nb, mr = std::min<int64_t>(q * LB, n - r1);  // rows of the blocks below
        if (mr <= 0) continue;
        if (w > 0 && (e = fl_dgemm(s, 0, 1, mr, nb, w, -1.0, A + r1 + k0 * lda, lda, A + j0 + k0 * lda, lda, 1.0,
                                   A + r1 + j0 * lda, lda)))
            return e;
        if ((e = fl_trsm_rlt(s, mr, nb, Ajj, lda, Linv + j * LB * LB, A + r1 + j0 * lda, lda, work))) return e;
    }
    return hipSuccess;
}

hipError_t fl_trtri_leaves(hipStream_t s, int64_t n, const double* L, int64_t ldl, double* Linv) {
    if (n <= 0) return hipSuccess;
    trtri_leaves_kernel<<<(unsigned)FL_DIV_UP(n, LB), LT, 0, s>>>(n, L, ldl, Linv);
    return hipGetLastError();
}

hipError_t fl_symmetrize(hipStream_t s, int64_t n, double* A, int64_t lda) {
    if (n <= 1) return hipSuccess;
    dim3 grid((unsigned)FL_DIV_UP(n, 256), (unsigned)(n < 65535 ? n : 65535));
    symmetrize_kernel<<<grid, 256, 0, s>>>(n, A, lda);
    return hipGetLastError();
}

int64_t fl_band_panel_elems(int64_t n, int64_t q) { return FL_DIV_UP(n, LB) * LB * (q + 1) * LB; }

// Panels of the strip-parallel banded solves (see band_solve_kernel): P is
// nbk panels of 128 x (q + 1) 128 (ld 128).  probs: device room for nbk
// GEMM descriptors.
hipError_t fl_band_panels(hipStream_t s, int64_t n, int64_t q, const double* L, int64_t ldl, const double* Linv,
                          double* P, int back, GemmProblem* probs) {
    if (n <= 0) return hipSuccess;
    const int64_t nbk = FL_DIV_UP(n, LB), KP = (q + 1) * LB;
    std::vector<GemmProblem> hp;
    for (int64_t i = 0; i < nbk; ++i) {
        const int64_t i0 = i * LB, nb = std::min<int64_t>(LB, n - i0);
        GemmProblem g{};
        if (!back) {
            const int64_t k0 = std::max<int64_t>(0, i - q) * LB, w = i0 - k0;
            if (w <= 0) continue;
            // -L_ii^-1 L_i,k: nb x w
            g.m = nb; g.n = w; g.k = nb;
            g.A = Linv + i * LB * LB; g.lda = LB;
            g.B = L + i0 + k0 * ldl; g.ldb = ldl;
        } else {
            const int64_t r1 = i0 + nb, w = std::min<int64_t>(q * LB, n - r1);
            if (w <= 0) continue;
            // -L_ii^-T L_k,i^T = -(L_ii^-1)^T (L_k,i)^T: nb x w
            g.m = nb; g.n = w; g.k = nb;
            g.A = Linv + i * LB * LB; g.lda = LB;
            g.B = L + r1 + i0 * ldl; g.ldb = ldl;
        }
        g.C = P + i * LB * KP + (back ? nb * LB : 0); g.ldc = LB;
        g.alpha = -1.0; g.beta = 0.0;
        hp.push_back(g);
    }
    hipError_t e;
    if (!hp.empty()) {
        if ((e = hipMemcpyAsync(probs, hp.data(), sizeof(GemmProblem) * hp.size(), hipMemcpyHostToDevice, s)))
            return e;
        if ((e = fl_dgemm_batched(s, back, back, probs, (int)hp.size(), LB, q * LB))) return e;
        // the descriptors live in host memory until the copy has been made
        if ((e = hipStreamSynchronize(s))) return e;
    }
    if (back)
        band_panel_diag_kernel<true><<<(unsigned)nbk, 256, 0, s>>>(n, q, Linv, P);
    else
        band_panel_diag_kernel<false><<<(unsigned)nbk, 256, 0, s>>>(n, q, Linv, P);
    return hipGetLastError();
}

// L X = B (back = 0) or L^T X = B (back = 1) for the banded factor, B n x m
// overwritten, from the panels of fl_band_panels.  bwb >= 0 (forward only):
// row r of B is zero beyond column r + bwb.
hipError_t fl_band_solve(hipStream_t s, int64_t n, int64_t q, const double* P, double* B, int64_t ldb, int64_t m,
                         int back, int64_t bwb) {
    if (n <= 0 || m <= 0) return hipSuccess;
    const unsigned grid = (unsigned)FL_DIV_UP(m, BSW);
    if (back)
        band_solve_kernel<true><<<grid, 256, 0, s>>>(n, q, P, B, ldb, m, -1);
    else
        band_solve_kernel<false><<<grid, 256, 0, s>>>(n, q, P, B, ldb, m, bwb);
    return hipGetLastError();
}
