// Many small generalized eigenproblems K phi = theta M phi (eq.
// discrete_laplace; the basis of each domain is computed once and reused,
// Section "Method") in ONE persistent launch.
//
// Every workgroup takes the next problem from an atomic counter over the
// problems sorted by n, largest first, and solves it alone, in FP64:
//   M = L L^T                      blocked Cholesky (32-column panels)
//   C = L^-1 (L^-1 K)^T            two blocked triangular solves
//   C = Q T Q^T                    Householder tridiagonalisation
//   T = Z_T diag(theta) Z_T^T      implicit QL with Wilkinson shifts; the
//                                  rotations of each sweep are staged in LDS
//                                  and applied to Z row-parallel
//   Z = Q Z_T                      block reflectors (I - V T V^T), 32 at a time
//   V = L^-T Z                     blocked triangular solve
// then theta ascending and V = [phi_1 .. phi_n], M-orthonormal.  The dense
// contractions use a register-tiled FP64 FMA tile (on gfx950 the FP64 vector
// rate equals the FP64 matrix-core rate).  No workgroup waits on another:
// the launch ends when the counter passes the last problem.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>
#include "internal.h"

namespace {

constexpr int BT = 512;                    // threads per workgroup (8 waves)
constexpr int NMAX = 1024;                 // largest problem
constexpr int PB = 32;                     // panel / reflector block width
constexpr int TM = 64, TN = 128, TK = 16;  // GEMM tile (4 x 4 outputs per thread)
constexpr int RPT = NMAX / BT;             // rows per thread in the tridiagonalisation
constexpr int QS = 4;                      // QL sweeps applied to Z per pass
static_assert(TM * TN == 16 * BT, "one 4 x 4 register tile per thread");
constexpr double EPS = 2.220446049250313e-16;

// The workgroup routines below are kept as separate (noinline) functions:
// fully inlined into the one persistent kernel, the register pressure (256
// VGPRs plus spills) produced wrong results in the blocked triangular solve
// at n > 32, while the same code called as functions, or in a small kernel,
// is exact.

struct BProb {
    int64_t n, ld;                                      // ld: of K, M and V
    const double* K;
    const double* M;
    double* V;
    double* theta;
    double* logtheta;
    double *L, *W, *A, *Z;                               // workspaces, ld n
    double* tau;                                        // n
};

struct Lds {
    double As[TK][TM + 1];
    double Bs[TK][TN + 1];
    double D[PB][PB + 1];
    double red[BT / 64];
    double va[2][NMAX];  // Householder vectors (two in flight), QL cosines
    double wa[2][NMAX];  // their w = p - (tau/2)(p^T v) v, QL sines
    double dd[NMAX];  // diagonal of T, then theta
    double ee[NMAX];  // off-diagonal of T
    double qx[2][NMAX];  // rotations of two more buffered QL sweeps
    double qy[2][NMAX];
    int rk[NMAX];     // ranks of theta
    int ival[4];
    int qlo[4], qhi[4];
    double dval[4];
};

// Barrier for data handed between the waves of the workgroup through global
// memory: drain this wave's stores, barrier, then drop stale vector-L1 lines.
// (A plain workgroup barrier on gfx950 waits for LDS traffic only: a store
// still in flight, or an L1 line fetched before another wave's store, could
// otherwise be read after it.)
__device__ inline void gsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ double wg_sum(double v, Lds& s) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s.red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < BT / 64; ++w) r += s.red[w];
    return r;
}

// C (m x n) = alpha op(A) op(B) + beta C, column-major, op = transpose when
// ta / tb.  C must not overlap A or B.
__device__ __attribute__((noinline)) void wg_gemm(bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int64_t lda,
                        const double* B, int64_t ldb, double beta, double* C, int64_t ldc, Lds& s) {
    if (m <= 0 || n <= 0) return;
    const int t = threadIdx.x;
    const int r0 = (t & 15) * 4, c0 = (t >> 4) * 4;
    const int tiles_m = (m + TM - 1) / TM, tiles_n = (n + TN - 1) / TN;
    for (int tile = 0; tile < tiles_m * tiles_n; ++tile) {
        const int i0 = (tile % tiles_m) * TM, j0 = (tile / tiles_m) * TN;
        double acc[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
        for (int k0 = 0; k0 < k; k0 += TK) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < (TM * TK) / BT; ++q) {
                const int e = t + BT * q;
                int i, kk;
                if (!ta) {
                    i = e % TM;
                    kk = e / TM;
                } else {
                    kk = e % TK;
                    i = e / TK;
                }
                const int gi = i0 + i, gk = k0 + kk;
                double a = 0.0;
                if (gi < m && gk < k) a = ta ? A[gk + (int64_t)gi * lda] : A[gi + (int64_t)gk * lda];
                s.As[kk][i] = a;
            }
#pragma unroll
            for (int q = 0; q < (TN * TK) / BT; ++q) {
                const int e = t + BT * q;
                int j, kb;
                if (!tb) {
                    kb = e % TK;
                    j = e / TK;
                } else {
                    j = e % TN;
                    kb = e / TN;
                }
                const int gj = j0 + j, gk2 = k0 + kb;
                double b = 0.0;
                if (gj < n && gk2 < k) b = tb ? B[gj + (int64_t)gk2 * ldb] : B[gk2 + (int64_t)gj * ldb];
                s.Bs[kb][j] = b;
            }
            __syncthreads();
#pragma unroll 4
            for (int kk = 0; kk < TK; ++kk) {
                double a[4], b[4];
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    a[x] = s.As[kk][r0 + x];
                    b[x] = s.Bs[kk][c0 + x];
                }
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
            }
        }
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int gj = j0 + c0 + y;
            if (gj >= n) continue;
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                const int gi = i0 + r0 + x;
                if (gi >= m) continue;
                double* cp = C + gi + (int64_t)gj * ldc;
                *cp = (beta == 0.0) ? alpha * acc[x][y] : alpha * acc[x][y] + beta * *cp;
            }
        }
    }
    gsync();
}

// Cholesky of the leading n x n of A (lower triangle used and overwritten).
// Returns 0, or the 1-based index of the first non-positive pivot.
__device__ __attribute__((noinline)) int wg_potrf(int n, double* A, int64_t lda, Lds& s) {
    const int t = threadIdx.x;
    for (int j0 = 0; j0 < n; j0 += PB) {
        const int jb = min(PB, n - j0);
        if (j0 > 0)
            wg_gemm(false, true, n - j0, jb, j0, -1.0, A + j0, lda, A + j0, lda, 1.0, A + j0 + (int64_t)j0 * lda,
                    lda, s);
        for (int e = t; e < jb * jb; e += BT) {
            const int r = e % jb, c = e / jb;
            s.D[r][c] = A[j0 + r + (int64_t)(j0 + c) * lda];
        }
        if (t == 0) s.ival[0] = 0;
        __syncthreads();
        for (int c = 0; c < jb; ++c) {
            if (t == 0) {
                double dcc = s.D[c][c];
                if (!(dcc > 0.0)) {
                    if (!s.ival[0]) s.ival[0] = j0 + c + 1;
                    dcc = 1.0;
                }
                s.D[c][c] = sqrt(dcc);
            }
            __syncthreads();
            if (t > c && t < jb) s.D[t][c] /= s.D[c][c];
            __syncthreads();
            for (int e = t; e < jb * jb; e += BT) {
                const int r = e % jb, q = e / jb;
                if (q > c && r >= q) s.D[r][q] -= s.D[r][c] * s.D[q][c];
            }
            __syncthreads();
        }
        const int bad = s.ival[0];
        if (bad) return bad;
        for (int e = t; e < jb * jb; e += BT) {
            const int r = e % jb, c = e / jb;
            if (r >= c) A[j0 + r + (int64_t)(j0 + c) * lda] = s.D[r][c];
        }
        // rows below the block: x L_jj^T = a
        for (int r = j0 + jb + t; r < n; r += BT) {
            double x[PB];
#pragma unroll
            for (int c = 0; c < PB; ++c) {
                if (c < jb) {
                    double v = A[r + (int64_t)(j0 + c) * lda];
#pragma unroll
                    for (int q = 0; q < c; ++q) v -= x[q] * s.D[c][q];
                    x[c] = v / s.D[c][c];
                    A[r + (int64_t)(j0 + c) * lda] = x[c];
                } else {
                    x[c] = 0.0;
                }
            }
        }
        gsync();
    }
    return 0;
}

// Solve L X = B in place (L lower, n x n; B n x nrhs).
__device__ __attribute__((noinline)) void wg_trsm_ln(int n, int nrhs, const double* L, int64_t ldl, double* B, int64_t ldb, Lds& s) {
    const int t = threadIdx.x;
    for (int i0 = 0; i0 < n; i0 += PB) {
        const int ib = min(PB, n - i0);
        for (int e = t; e < PB * PB; e += BT) {
            const int r = e % PB, c = e / PB;
            s.D[r][c] = (r < ib && c <= r) ? L[i0 + r + (int64_t)(i0 + c) * ldl] : 0.0;
        }
        __syncthreads();
        for (int j = t; j < nrhs; j += BT) {
            double x[PB];
#pragma unroll
            for (int r = 0; r < PB; ++r) {
                if (r < ib) {
                    double v = B[i0 + r + (int64_t)j * ldb];
#pragma unroll
                    for (int q = 0; q < r; ++q) v -= s.D[r][q] * x[q];
                    x[r] = v / s.D[r][r];
                    B[i0 + r + (int64_t)j * ldb] = x[r];
                } else {
                    x[r] = 0.0;
                }
            }
        }
        gsync();
        if (i0 + ib < n)
            wg_gemm(false, false, n - i0 - ib, nrhs, ib, -1.0, L + i0 + ib + (int64_t)i0 * ldl, ldl, B + i0, ldb,
                    1.0, B + i0 + ib, ldb, s);
    }
}

// Solve L^T X = B in place.
__device__ __attribute__((noinline)) void wg_trsm_lt(int n, int nrhs, const double* L, int64_t ldl, double* B, int64_t ldb, Lds& s) {
    const int t = threadIdx.x;
    const int nblk = (n + PB - 1) / PB;
    for (int bi = nblk - 1; bi >= 0; --bi) {
        const int i0 = bi * PB, ib = min(PB, n - i0);
        for (int e = t; e < PB * PB; e += BT) {
            const int r = e % PB, c = e / PB;
            s.D[r][c] = (r < ib && c <= r) ? L[i0 + r + (int64_t)(i0 + c) * ldl] : 0.0;
        }
        __syncthreads();
        for (int j = t; j < nrhs; j += BT) {
            double x[PB];
#pragma unroll
            for (int r = PB - 1; r >= 0; --r) {
                if (r < ib) {
                    double v = B[i0 + r + (int64_t)j * ldb];
#pragma unroll
                    for (int q = r + 1; q < PB; ++q)
                        if (q < ib) v -= s.D[q][r] * x[q];
                    x[r] = v / s.D[r][r];
                    B[i0 + r + (int64_t)j * ldb] = x[r];
                } else {
                    x[r] = 0.0;
                }
            }
        }
        gsync();
        if (i0 > 0) wg_gemm(true, false, i0, nrhs, ib, -1.0, L + i0, ldl, B + i0, ldb, 1.0, B, ldb, s);
    }
}

// In the tridiagonalisation thread t owns the global rows g = t + q BT
// (q < RPT) of A for the whole reduction, so every element of A is read and
// written by one thread only and only LDS carries data between threads.

// Householder reflector of x = A[g0 : g0 + m, c] (x[0] = alpha at row g0):
// x[1:] is scaled in place into v[1:] (also copied to the LDS vector v,
// indexed from row g0).  Returns tau; beta goes to *beta.
__device__ double wg_house(int n, int64_t g0, int m, double* col, double alpha, double* v, double* beta,
                           Lds& s) {
    const int t = threadIdx.x;
    double loc = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t g = t + q * BT;
        const int64_t r = g - g0;
        if (g < n && r >= 1 && r < m) loc += col[g] * col[g];
    }
    const double xn2 = wg_sum(loc, s);
    double tk = 0.0, bt = alpha;
    const double sc = (xn2 > 0.0) ? 1.0 / (alpha - (-copysign(sqrt(alpha * alpha + xn2), alpha))) : 0.0;
    if (xn2 > 0.0) {
        bt = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tk = (bt - alpha) / bt;
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t g = t + q * BT;
        const int64_t r = g - g0;
        if (g < n && r >= 1 && r < m) {
            const double vr = col[g] * sc;
            col[g] = vr;
            v[r] = vr;
        }
    }
    if (t == 0) v[0] = 1.0;
    *beta = bt;
    return tk;
}

// w = p - (tau/2)(p^T v) v with p = tau acc; acc[q] belongs to global row
// t + q BT = trailing row i + g0.
__device__ void wg_make_w(int n, int64_t g0, int m, double tk, const double (&acc)[RPT], const double* v, double* w,
                          Lds& s) {
    const int t = threadIdx.x;
    double loc = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t i = t + q * BT - g0;
        if (i >= 0 && i < m) loc += tk * acc[q] * v[i];
    }
    const double hc = 0.5 * tk * wg_sum(loc, s);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t i = t + q * BT - g0;
        if (i >= 0 && i < m) w[i] = tk * acc[q] - hc * v[i];
    }
    __syncthreads();
}

// Householder tridiagonalisation of the symmetric A (full storage, kept
// exactly symmetric), lower reflectors: reflector k has v = (1, A[k+2:n, k])
// on rows k+1..n-1 and tau[k]; d and e (e[i] couples i and i+1) are left in
// s.dd and s.ee.  One pass over the trailing matrix per step: the rank-2
// update of step k, A22 -= v w^T + w v^T, is fused with the product
// A22' v' of step k+1 (A22' = A22 without its first row and column).
__device__ __attribute__((noinline)) void wg_sytrd(int n, double* A, int64_t lda, double* tau, Lds& s) {
    const int t = threadIdx.x;
    if (n <= 2) {
        if (t == 0) {
            s.dd[0] = A[0];
            if (n == 2) {
                s.dd[1] = A[1 + lda];
                s.ee[0] = A[1];
            }
            s.ee[n - 1] = 0.0;
        }
        __syncthreads();
        return;
    }
    // reflector 0 (column 0, rows 1..n-1) and acc = A[1:, 1:] v
    {
        double beta;
        if (t == 0) s.dval[1] = A[1];
        __syncthreads();
        const double tk = wg_house(n, 1, n - 1, A, s.dval[1], s.va[0], &beta, s);
        if (t == 0) {
            s.dd[0] = A[0];
            s.ee[0] = beta;
            tau[0] = tk;
        }
        __syncthreads();
        double acc[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) acc[q] = 0.0;
        for (int j = 1; j < n; ++j) {
            const double vj = s.va[0][j - 1];
            const double* col = A + (int64_t)j * lda;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int g = t + q * BT;
                if (g >= 1 && g < n) acc[q] = fma(col[g], vj, acc[q]);
            }
        }
        wg_make_w(n, 1, n - 1, tk, acc, s.va[0], s.wa[0], s);
    }
    for (int k = 0; k < n - 2; ++k) {
        const int cur = k & 1, nxt = cur ^ 1;
        const double* v = s.va[cur];  // step k, indexed by trailing row: global row k+1+i
        const double* w = s.wa[cur];
        const int64_t g0 = k + 1;      // first global row (and column) of A22
        const int m = n - k - 1;       // order of A22
        if (k + 1 < n - 2) {
            // (a) column g0 (rows g0..n-1) with step k's update: d[k+1], and x of step k+1
            double* c0 = A + g0 * lda;
            const double v0 = v[0], w0 = w[0];
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int64_t g = t + q * BT;
                const int64_t i = g - g0;
                if (g < n && i >= 0) {
                    const double p1 = __dmul_rn(v[i], w0), p2 = __dmul_rn(w[i], v0);
                    c0[g] = __dsub_rn(c0[g], __dadd_rn(p1, p2));
                    if (i == 0) s.dval[0] = c0[g];
                    if (i == 1) s.dval[1] = c0[g];
                }
            }
            __syncthreads();
            // (b) reflector k+1 from rows g0+1.. of that column
            double beta;
            const double tk = wg_house(n, g0 + 1, m - 1, c0, s.dval[1], s.va[nxt], &beta, s);
            if (t == 0) {
                s.dd[k + 1] = s.dval[0];
                s.ee[k + 1] = beta;
                tau[k + 1] = tk;
            }
            __syncthreads();
            // (c) rows/columns g0+1.. : A -= v w^T + w v^T, fused with acc = A v'
            const double* v2 = s.va[nxt];  // indexed from global row g0+1
            double acc[RPT];
#pragma unroll
            for (int q = 0; q < RPT; ++q) acc[q] = 0.0;
            for (int j = 1; j < m; ++j) {
                const double vj = v[j], wj = w[j], v2j = v2[j - 1];
                double* col = A + (g0 + j) * lda;
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    const int64_t g = t + q * BT;
                    const int64_t i = g - g0;
                    if (g < n && i >= 1) {
                        const double p1 = __dmul_rn(v[i], wj), p2 = __dmul_rn(w[i], vj);
                        const double a = __dsub_rn(col[g], __dadd_rn(p1, p2));
                        col[g] = a;
                        acc[q] = fma(a, v2j, acc[q]);
                    }
                }
            }
            // (d) w of step k+1
            wg_make_w(n, g0 + 1, m - 1, tk, acc, v2, s.wa[nxt], s);
        } else {
            // last step (m == 2): the remaining 2 x 2 block, rows n-2 and n-1
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int64_t g = t + q * BT;
                const int64_t i = g - g0;
                if (g < n && i >= 0) {
                    for (int j = 0; j <= i; ++j) {
                        const double p1 = __dmul_rn(v[i], w[j]), p2 = __dmul_rn(w[i], v[j]);
                        double* a = A + g + (g0 + j) * lda;
                        *a = __dsub_rn(*a, __dadd_rn(p1, p2));
                    }
                    if (i == 0) s.dd[n - 2] = A[g + g0 * lda];
                    if (i == 1) {
                        s.ee[n - 2] = A[g + g0 * lda];
                        s.dd[n - 1] = A[g + (g0 + 1) * lda];
                    }
                }
            }
            if (t == 0) s.ee[n - 1] = 0.0;
            __syncthreads();
        }
    }
}

__device__ inline double* ql_cos(Lds& s, int b) { return b < 2 ? s.va[b] : s.qx[b - 2]; }
__device__ inline double* ql_sin(Lds& s, int b) { return b < 2 ? s.wa[b] : s.qy[b - 2]; }

// Apply nb <= QS buffered QL sweeps to the rows of Z in one pass.  Sweep b
// applies its rotations (i, i+1), i = hi_b .. lo_b, in that order.  Each row is
// walked downwards with a register window of 2 QS columns: at position c,
// sweep b rotates columns (c + 2b, c + 2b + 1).  Sweep b at i needs sweep b-1
// to have rotated (i-1, i), which happened at position c + 1, and nothing
// touches column c + 2 QS - 1 after position c, so it is written back then.
__device__ void ql_apply(int n, double* Z, int64_t ldz, int nb, Lds& s) {
    const int t = threadIdx.x;
    int lo[QS], hi[QS];
    const double* C[QS];
    const double* S[QS];
    int cstart = -(1 << 30), cend = 1 << 30;
#pragma unroll
    for (int b = 0; b < QS; ++b) {
        lo[b] = (b < nb) ? s.qlo[b] : 1;
        hi[b] = (b < nb) ? s.qhi[b] : 0;
        C[b] = ql_cos(s, b);
        S[b] = ql_sin(s, b);
        if (lo[b] <= hi[b]) {
            cstart = max(cstart, hi[b] - 2 * b);
            cend = min(cend, lo[b] - 2 * b);
        }
    }
    if (cstart < cend) return;  // no rotations (uniform: every thread read the same LDS)
    for (int row = t; row < n; row += BT) {
        double* zr = Z + row;
        double win[2 * QS];
#pragma unroll
        for (int k = 0; k < 2 * QS; ++k) {
            const int col = cstart + k;
            win[k] = (col >= 0 && col < n) ? zr[(int64_t)col * ldz] : 0.0;
        }
        int c = cstart;
        while (c >= cend) {
            const int cnt = min(8, c - cend + 1);
            double pre[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int col = c - 1 - q;
                pre[q] = (q < cnt && col >= 0) ? zr[(int64_t)col * ldz] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (q < cnt) {
                    const int cc = c - q;
#pragma unroll
                    for (int b = 0; b < QS; ++b) {
                        const int i = cc + 2 * b;
                        if (lo[b] <= i && i <= hi[b]) {
                            const double cs = C[b][i], sn = S[b][i];
                            const double x = win[2 * b], y = win[2 * b + 1];
                            win[2 * b] = cs * x - sn * y;
                            win[2 * b + 1] = sn * x + cs * y;
                        }
                    }
                    const int col_out = cc + 2 * QS - 1;
                    if (col_out < n) zr[(int64_t)col_out * ldz] = win[2 * QS - 1];
#pragma unroll
                    for (int k = 2 * QS - 1; k > 0; --k) win[k] = win[k - 1];
                    win[0] = pre[q];
                }
            }
            c -= cnt;
        }
        // the window now holds columns cend-1 .. cend-1 + 2QS-1
#pragma unroll
        for (int k = 0; k < 2 * QS; ++k) {
            const int col = cend - 1 + k;
            if (col >= 0 && col < n) zr[(int64_t)col * ldz] = win[k];
        }
    }
}

// Implicit QL with Wilkinson shifts on (s.dd, s.ee); Z (n x n, identity on
// entry) accumulates the rotations.  One thread runs each sweep's scalar
// recurrence and stages its rotations in LDS; every QS sweeps all threads
// apply them to their rows of Z in one pass.  Returns 0, or l+1 if
// eigenvalue l took over 60 sweeps.
__device__ __attribute__((noinline)) int wg_steql(int n, double* Z, int64_t ldz, Lds& s) {
    const int t = threadIdx.x;
    int nb = 0;  // buffered sweeps (the same in every thread)
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            if (t == 0) {
                int mm = l;
                for (; mm < n - 1; ++mm) {
                    const double dd = fabs(s.dd[mm]) + fabs(s.dd[mm + 1]);
                    if (fabs(s.ee[mm]) <= EPS * dd) break;
                }
                s.ival[1] = mm;
            }
            __syncthreads();
            const int m = s.ival[1];
            __syncthreads();
            if (m == l) break;
            if (++iter > 60) return l + 1;
            if (t == 0) {
                double* qc = ql_cos(s, nb);
                double* qs = ql_sin(s, nb);
                // shift from the leading 2 x 2 of the unreduced block [l, m]
                double g = (s.dd[l + 1] - s.dd[l]) / (2.0 * s.ee[l]);
                double r = hypot(g, 1.0);
                g = s.dd[m] - s.dd[l] + s.ee[l] / (g + copysign(r, g));
                double sn = 1.0, c = 1.0, p = 0.0;
                int i = m - 1;
                bool early = false;
                // the chain is latency bound: d and e of the next step are read
                // ahead, and one square root and one reciprocal replace hypot and
                // two divisions (|f|, |g| stay far from overflow for these pencils)
                double ei = s.ee[i], di = s.dd[i], di1 = s.dd[i + 1];
                for (; i >= l; --i) {
                    const double ein = (i > l) ? s.ee[i - 1] : 0.0;
                    const double din = (i > l) ? s.dd[i - 1] : 0.0;
                    const double f = sn * ei, b = c * ei;
                    r = sqrt(f * f + g * g);
                    s.ee[i + 1] = r;
                    if (r == 0.0) {  // the block splits: restart on it
                        s.dd[i + 1] = di1 - p;
                        s.ee[m] = 0.0;
                        early = true;
                        break;
                    }
                    const double inv = 1.0 / r;
                    sn = f * inv;
                    c = g * inv;
                    g = di1 - p;
                    r = (di - g) * sn + 2.0 * c * b;
                    p = sn * r;
                    s.dd[i + 1] = g + p;
                    g = c * r - b;
                    qc[i] = c;
                    qs[i] = sn;
                    ei = ein;
                    di1 = di;
                    di = din;
                }
                if (!early) {
                    s.dd[l] -= p;
                    s.ee[l] = g;
                    s.ee[m] = 0.0;
                    s.qlo[nb] = l;
                } else {
                    s.qlo[nb] = i + 1;
                }
                s.qhi[nb] = m - 1;
            }
            __syncthreads();
            if (++nb == QS) {
                ql_apply(n, Z, ldz, nb, s);
                nb = 0;
                __syncthreads();
            }
        }
    }
    if (nb) ql_apply(n, Z, ldz, nb, s);
    __syncthreads();
    return 0;
}

// Z := Q Z with Q = H_0 H_1 ... H_{n-3} from wg_sytrd, applied as block
// reflectors of PB consecutive H (forward, columnwise: I - V T V^T), last
// block first.  work: >= 3 PB n + PB PB doubles.
__device__ __attribute__((noinline)) void wg_ormtr(int n, const double* A, int64_t lda, const double* tau, double* Z, int64_t ldz,
                         double* work, Lds& s) {
    const int t = threadIdx.x;
    const int nref = n - 2;
    if (nref <= 0) return;
    const int nblk = (nref + PB - 1) / PB;
    for (int bi = nblk - 1; bi >= 0; --bi) {
        const int k0 = bi * PB, nb = min(PB, nref - k0);
        const int rows = n - k0 - 1;  // rows k0+1 .. n-1
        double* Vb = work;                          // rows x nb
        double* Tm = Vb + (int64_t)rows * PB;       // PB x PB
        double* Wt = Tm + PB * PB;                  // nb x n
        double* Wt2 = Wt + (int64_t)PB * n;         // nb x n
        for (int c = 0; c < nb; ++c)
            for (int rr = t; rr < rows; rr += BT)
                Vb[rr + (int64_t)c * rows] =
                    rr < c ? 0.0 : (rr == c ? 1.0 : A[(k0 + 1 + rr) + (int64_t)(k0 + c) * lda]);
        gsync();
        // G = V^T V (in Wt), then T column by column: T[c][c] = tau_c,
        // T[0:c, c] = -tau_c T[0:c, 0:c] G[0:c, c]
        wg_gemm(true, false, nb, nb, rows, 1.0, Vb, rows, Vb, rows, 0.0, Wt, PB, s);
        for (int e = t; e < PB * PB; e += BT) s.D[e % PB][e / PB] = 0.0;
        __syncthreads();
        for (int c = 0; c < nb; ++c) {
            const double tc = tau[k0 + c];
            double acc = 0.0;
            if (t < c) {
                for (int q = t; q < c; ++q) acc += s.D[t][q] * Wt[q + c * PB];
            }
            __syncthreads();
            if (t < c) s.D[t][c] = -tc * acc;
            if (t == c) s.D[c][c] = tc;
            __syncthreads();
        }
        for (int e = t; e < PB * PB; e += BT) Tm[e] = s.D[e % PB][e / PB];
        gsync();
        wg_gemm(true, false, nb, n, rows, 1.0, Vb, rows, Z + k0 + 1, ldz, 0.0, Wt, nb, s);
        wg_gemm(false, false, nb, n, nb, 1.0, Tm, PB, Wt, nb, 0.0, Wt2, nb, s);
        wg_gemm(false, false, rows, n, nb, -1.0, Vb, rows, Wt2, nb, 1.0, Z + k0 + 1, ldz, s);
    }
}

__device__ int64_t solve_one(const BProb& p, Lds& s) {
    const int t = threadIdx.x;
    const int n = (int)p.n;
    const int64_t ld = p.ld;
    double *L = p.L, *W = p.W, *A = p.A, *Z = p.Z;
    for (int j = 0; j < n; ++j)
        for (int i = t; i < n; i += BT) {
            L[i + (int64_t)j * n] = p.M[i + j * ld];
            W[i + (int64_t)j * n] = p.K[i + j * ld];
        }
    gsync();
    const int piv = wg_potrf(n, L, n, s);
    if (piv) return piv;
    wg_trsm_ln(n, n, L, n, W, n, s);  // W = L^-1 K
    for (int j = 0; j < n; ++j)
        for (int i = t; i < n; i += BT) A[i + (int64_t)j * n] = W[j + (int64_t)i * n];
    gsync();
    wg_trsm_ln(n, n, L, n, A, n, s);  // A = L^-1 K L^-T
    for (int j = 0; j < n; ++j)
        for (int i = j + 1 + t; i < n; i += BT) {
            const double v = 0.5 * (A[i + (int64_t)j * n] + A[j + (int64_t)i * n]);
            A[i + (int64_t)j * n] = v;
            A[j + (int64_t)i * n] = v;
        }
    gsync();
    wg_sytrd(n, A, n, p.tau, s);
    for (int j = 0; j < n; ++j)
        for (int i = t; i < n; i += BT) Z[i + (int64_t)j * n] = (i == j) ? 1.0 : 0.0;
    gsync();
    const int ql = wg_steql(n, Z, n, s);
    gsync();
    if (ql) return -(int64_t)ql;
    wg_ormtr(n, A, n, p.tau, Z, n, W, s);
    wg_trsm_lt(n, n, L, n, Z, n, s);  // V = L^-T Z
    for (int i = t; i < n; i += BT) {
        const double di = s.dd[i];
        int r = 0;
        for (int j = 0; j < n; ++j) {
            const double dj = s.dd[j];
            r += (dj < di || (dj == di && j < i)) ? 1 : 0;
        }
        s.rk[i] = r;
        p.theta[r] = di;
        p.logtheta[r] = log(di);
    }
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        const int dst = s.rk[j];
        for (int i = t; i < n; i += BT) p.V[i + (int64_t)dst * ld] = Z[i + (int64_t)j * n];
    }
    __syncthreads();
    return 0;
}

__global__ __launch_bounds__(BT) void batched_eig_kernel(const BProb* __restrict__ probs, const int* __restrict__ order,
                                                         int count, unsigned* next, int64_t* status) {
    __shared__ Lds s;
    for (;;) {
        if (threadIdx.x == 0) s.ival[0] = (int)atomicAdd(next, 1u);
        __syncthreads();
        const int q = s.ival[0];
        __syncthreads();
        if (q >= count) break;
        const int pi = order[q];
        const int64_t st = solve_one(probs[pi], s);
        if (threadIdx.x == 0) status[pi] = st;
        __syncthreads();
    }
}

}  // namespace

extern "C" int fl_eigensolve_batched(fl_ctx* ctx, int64_t count, fl_op* const* ops, int precision,
                                     fl_eig_info* infos) {
    if (!ctx) return FL_EINVAL;
    if (count < 0 || (count > 0 && !ops)) return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_batched: bad arguments");
    if (precision != FL_FP64)
        return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_batched: the batched solver runs in FP64 only");
    if (count == 0) return FL_OK;
    if (count > (int64_t)1 << 30) return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_batched: too many problems");
    for (int64_t i = 0; i < count; ++i) {
        const fl_op* op = ops[i];
        if (!op || op->device != ctx->device)
            return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_batched: null operator or operator of another device");
        if (op->n < 1 || op->n > NMAX)
            return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_batched: each n must be in [1, 1024]");
        for (int64_t j = 0; j < i; ++j)
            if (ops[j] == op) return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_batched: an operator appears twice");
    }
    FL_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    // workspace: L, W, A, Z and tau per problem, 256-byte aligned
    std::vector<int64_t> off(count);
    int64_t tot = 0;
    auto al = [](int64_t x) { return (x + 31) / 32 * 32; };
    for (int64_t i = 0; i < count; ++i) {
        const int64_t n = ops[i]->n;
        const int64_t wsz = std::max<int64_t>(n * n, 3 * (int64_t)PB * n + PB * PB);
        off[i] = tot;
        tot += al(n * n) * 3 + al(wsz) + al(n);
    }
    DevBuf bws, bprobs, border, bnext, bstat;
    FL_HIP(ctx, bws.alloc(sizeof(double) * tot));
    std::vector<BProb> hp(count);
    for (int64_t i = 0; i < count; ++i) {
        fl_op* op = ops[i];
        const int64_t n = op->n;
        if (!op->theta) FL_HIP(ctx, hipMalloc(&op->theta, sizeof(double) * n));
        if (!op->logtheta) FL_HIP(ctx, hipMalloc(&op->logtheta, sizeof(double) * n));
        if (!op->V) FL_HIP(ctx, hipMalloc(&op->V, sizeof(double) * op->ld * n));
        op->has_eig = 0;
        double* w = bws.as<double>() + off[i];
        const int64_t wsz = std::max<int64_t>(n * n, 3 * (int64_t)PB * n + PB * PB);
        BProb& b = hp[i];
        b.n = n;
        b.ld = op->ld;
        b.K = op->K;
        b.M = op->M;
        b.V = op->V;
        b.theta = op->theta;
        b.logtheta = op->logtheta;
        b.L = w;
        b.A = w + al(n * n);
        b.Z = w + 2 * al(n * n);
        b.W = w + 3 * al(n * n);
        b.tau = b.W + al(wsz);
    }
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ops[a]->n > ops[b]->n; });
    FL_HIP(ctx, bprobs.alloc(sizeof(BProb) * count));
    FL_HIP(ctx, border.alloc(sizeof(int) * count));
    FL_HIP(ctx, bnext.alloc(sizeof(unsigned)));
    FL_HIP(ctx, bstat.alloc(sizeof(int64_t) * count));
    FL_HIP(ctx, hipMemcpyAsync(bprobs.p, hp.data(), sizeof(BProb) * count, hipMemcpyHostToDevice, s));
    FL_HIP(ctx, hipMemcpyAsync(border.p, order.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
    FL_HIP(ctx, hipMemsetAsync(bnext.p, 0, sizeof(unsigned), s));
    FL_HIP(ctx, hipMemsetAsync(bstat.p, 0, sizeof(int64_t) * count, s));
    int cus = 256;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) cus = prop.multiProcessorCount;
    }
    const unsigned grid = (unsigned)std::min<int64_t>(count, 2 * (int64_t)cus);
    hipEvent_t e0, e1;
    FL_HIP(ctx, hipEventCreate(&e0));
    FL_HIP(ctx, hipEventCreate(&e1));
    FL_HIP(ctx, hipEventRecord(e0, s));
    {
        KScope ks("batched_eig", s);
        batched_eig_kernel<<<grid, BT, 0, s>>>(bprobs.as<BProb>(), border.as<int>(), (int)count, bnext.as<unsigned>(),
                                               bstat.as<int64_t>());
    }
    hipError_t le = hipGetLastError();
    FL_HIP(ctx, hipEventRecord(e1, s));
    std::vector<int64_t> st(count);
    FL_HIP(ctx, hipMemcpyAsync(st.data(), bstat.p, sizeof(int64_t) * count, hipMemcpyDeviceToHost, s));
    FL_HIP(ctx, hipStreamSynchronize(s));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    FL_HIP(ctx, le);
    int rc = FL_OK;
    for (int64_t i = 0; i < count; ++i) {
        int code = FL_OK;
        if (st[i] > 0) code = FL_ENOTSPD;
        if (st[i] < 0) code = FL_ENOCONV;
        if (code == FL_OK) ops[i]->has_eig = 1;
        if (infos) {
            infos[i] = fl_eig_info{};
            infos[i].status = code;
            infos[i].index = st[i] > 0 ? st[i] : (st[i] < 0 ? -st[i] : 0);
            infos[i].total_ms = ms;
            const double n = (double)ops[i]->n;
            infos[i].flops_nominal = 9.0 * n * n * n;
        }
        if (code != FL_OK && rc == FL_OK) {
            rc = code;
            fl_fail(ctx, code,
                    std::string("fl_eigensolve_batched: problem ") + std::to_string(i) +
                        (code == FL_ENOTSPD ? ": M is not positive definite at pivot "
                                            : ": QL did not converge at eigenvalue ") +
                        std::to_string(st[i] > 0 ? st[i] : -st[i]));
        }
    }
    return rc;
}
