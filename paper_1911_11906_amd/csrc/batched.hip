// Many small generalized eigenproblems K phi = theta M phi (eq.
// discrete_laplace; the basis of each domain is computed once and reused,
// Section "Method") in ONE persistent launch.
//
// Every workgroup takes the next problem from an atomic counter over the
// problems sorted by n, largest first, and solves it alone, in FP64:
//   M = L L^T                      blocked Cholesky (32-column panels)
//   C = L^-1 (L^-1 K)^T            two blocked triangular solves
//   C = Q T Q^T                    Householder tridiagonalisation
//   T = Z_T diag(theta) Z_T^T      divide and conquer: leaves of <= 32 by
//                                  implicit QL (one wave each, in LDS), merges
//                                  by secular equations and two GEMMs
//   Z = Q Z_T                      block reflectors (I - V T V^T), 32 at a time
//   V = L^-T Z                     blocked triangular solve
// then theta ascending and V = [phi_1 .. phi_n], M-orthonormal.  The dense
// contractions run on the FP64 matrix cores (v_mfma_f64_16x16x4f64: eight
// waves of 32 x 32 over a 64 x 128 workgroup tile, k-slabs of 32 staged in
// LDS).  No workgroup waits on another: the launch ends when the counter
// passes the last problem.
#include <algorithm>
#include <memory>
#include <cmath>
#include <numeric>
#include <vector>
#include "internal.h"

namespace {

constexpr int BT = 512;                    // threads per workgroup (8 waves)
constexpr int NMAX = 1024;                 // largest problem
constexpr int PB = 32;                     // panel / reflector block width
constexpr int OB = 128;                    // row group of the two-level triangular solves
constexpr int TM = 64, TN = 128, TK = 32;  // GEMM tile: eight waves of 32 x 32, k-slab 32
constexpr int RPT = NMAX / BT;             // rows per thread in the tridiagonalisation
constexpr int DCL = 32;                    // largest leaf of the divide and conquer
constexpr int SU = 8;                      // columns per chunk in the tridiagonalisation's update
constexpr double EPS = 2.220446049250313e-16;

// The workgroup routines below are separate (noinline) functions: fully
// inlined into the persistent kernel they run no faster (same launch time on
// the 256-problem batch) and the code is several times larger.  (An earlier
// version, with generic pointers for global memory, gave wrong triangular
// solves at n > 32 when fully inlined; the current code, global accesses
// through address-space-1 pointers, passes every batched check either way.)

struct BProb {
    int64_t n, ld;                                      // ld: of K, M and V
    int64_t bw;                                         // half-bandwidth of M (n - 1: dense)
    const double* K;
    const double* M;
    double* V;
    double* theta;
    double* logtheta;
    double *L, *W, *A, *Z;                               // workspaces, ld n
    double *U, *Y;                                      // divide and conquer work, n x n
    double* R;                                          // 4 n
    double* tau;                                        // n
};

struct Lds {
    double As[TK][TM + 1];
    double Bs[TK][TN + 1];
    double D[PB][PB + 1];
    double red[BT / 64];
    double va[2][NMAX];  // Householder vectors (two in flight); divide and conquer scratch
    double wa[2][NMAX];  // their w = p - (tau/2)(p^T v) v
    double dd[NMAX];  // diagonal of T, then theta
    double ee[NMAX];  // off-diagonal of T
    double qx[2][NMAX];  // divide and conquer scratch
    double qy[2][NMAX];
    int rk[NMAX];     // ranks of theta
    int ix[NMAX];     // divide and conquer: deflated columns
    double lq[BT / 64][4][DCL];  // divide and conquer leaves: d, e, cosines, sines per wave
    int lb[NMAX / DCL + 2];      // leaf boundaries
    int ival[4];
    int qlo[4], qhi[4];
    double dval[4];
};

// Barrier for data handed between the waves of the workgroup through global
// memory: drain this wave's stores, barrier, then drop stale vector-L1 lines.
// (A plain workgroup barrier on gfx950 waits for LDS traffic only: a store
// still in flight, or an L1 line fetched before another wave's store, could
// otherwise be read after it.)
// Global memory seen as such.  A generic pointer makes every access a flat
// one; flat accesses may complete out of order with respect to LDS ones, so
// while any is in flight the compiler can only wait for all loads (and LDS
// reads) at once, and a prefetch no longer overlaps the work before it.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) int gint;

// Compiler-only barrier at the top of a per-thread loop over right-hand
// sides: the LDS block it reads is the same in every iteration, and hoisted
// out of the loop it would take the whole block into registers (and spill).
__device__ inline void keep_lds_reads_here() { __asm__ volatile("" ::: "memory"); }

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
// ta / tb.  C must not overlap A or B.  Tiles of 64 x 128 on the FP64
// matrix cores (v_mfma_f64_16x16x4f64): wave w owns the 32 x 32 block
// (w % 2, w / 2); the MFMA "A" operand is fed from op(B) and "B" from op(A),
// so accumulator register r of lane l holds C[16 ti + l % 16][16 tj + l / 16
// + 4 r] and the 16 lanes of a row group store consecutive rows.  The next
// k-slab is loaded into registers (unconditionally, indices clamped into the
// operands) while the current one is multiplied from LDS.
__device__ __attribute__((noinline)) void wg_gemm(bool ta, bool tb, int m, int n, int k, double alpha, const double* Ag, int64_t lda,
                        const double* Bg, int64_t ldb, double beta, double* Cg, int64_t ldc, Lds& s) {
    if (m <= 0 || n <= 0) return;
    const gdouble* A = (const gdouble*)Ag;
    const gdouble* B = (const gdouble*)Bg;
    gdouble* C = (gdouble*)Cg;
    constexpr int NA = TM * TK / BT, NB = TN * TK / BT;
    static_assert(NA * BT == TM * TK && NB * BT == TN * TK && BT == 512, "eight waves, 64 x 128 tiles");
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int lr = lane >> 4, lc = lane & 15;
    const int wi = wave & 1, wj = wave >> 1;
    const int tiles_m = (m + TM - 1) / TM, tiles_n = (n + TN - 1) / TN;
    for (int tile = 0; tile < tiles_m * tiles_n; ++tile) {
        const int i0 = (tile % tiles_m) * TM, j0 = (tile / tiles_m) * TN;
        d4_t acc[2][2];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) acc[x][y] = d4_t{0, 0, 0, 0};
        double ra[NA], rb[NB];
        unsigned okm = 0;  // validity of the loaded elements, applied when staged
        auto gload = [&](int k0) {
            okm = 0;
#pragma unroll
            for (int q = 0; q < NA; ++q) {
                const int e = t + BT * q;
                const int i = ta ? e / TK : e % TM, kk = ta ? e % TK : e / TM;
                const int gi = i0 + i, gk = k0 + kk;
                okm |= (gi < m && gk < k ? 1u : 0u) << q;
                const int ci = gi < m ? gi : m - 1, ck = gk < k ? gk : k - 1;
                ra[q] = ta ? A[ck + (int64_t)ci * lda] : A[ci + (int64_t)ck * lda];
            }
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int e = t + BT * q;
                const int j = tb ? e % TN : e / TK, kb = tb ? e / TN : e % TK;
                const int gj = j0 + j, gk = k0 + kb;
                okm |= (gj < n && gk < k ? 1u : 0u) << (NA + q);
                const int cj = gj < n ? gj : n - 1, ck = gk < k ? gk : k - 1;
                rb[q] = tb ? B[cj + (int64_t)ck * ldb] : B[ck + (int64_t)cj * ldb];
            }
        };
        if (k > 0) gload(0);
        for (int k0 = 0; k0 < k; k0 += TK) {
            __syncthreads();  // the previous slab has been consumed
#pragma unroll
            for (int q = 0; q < NA; ++q) {
                const int e = t + BT * q;
                s.As[ta ? e % TK : e / TM][ta ? e / TK : e % TM] = ((okm >> q) & 1u) ? ra[q] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int e = t + BT * q;
                s.Bs[tb ? e / TN : e % TK][tb ? e % TN : e / TK] = ((okm >> (NA + q)) & 1u) ? rb[q] : 0.0;
            }
            __syncthreads();
            if (k0 + TK < k) gload(k0 + TK);
#pragma unroll
            for (int k4 = 0; k4 < TK; k4 += 4) {
                double fa[2], fb[2];
#pragma unroll
                for (int x = 0; x < 2; ++x) {
                    fa[x] = s.Bs[k4 + lr][wj * 32 + 16 * x + lc];
                    fb[x] = s.As[k4 + lr][wi * 32 + 16 * x + lc];
                }
#pragma unroll
                for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 2; ++tj)
                        acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[tj], fb[ti], acc[ti][tj], 0, 0, 0);
            }
        }
        // C: the 16 old values of this lane (clamped into C, unconditional)
        // loaded together before any store, then the valid ones written
        double cold[2][2][4];
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int tj = 0; tj < 2; ++tj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gi = min(i0 + wi * 32 + 16 * ti + lc, m - 1);
                    const int gj = min(j0 + wj * 32 + 16 * tj + lr + 4 * r, n - 1);
                    cold[ti][tj][r] = (beta == 0.0) ? 0.0 : C[gi + (int64_t)gj * ldc];
                }
#pragma unroll
        for (int ti = 0; ti < 2; ++ti) {
            const int gi = i0 + wi * 32 + 16 * ti + lc;
            if (gi >= m) continue;
#pragma unroll
            for (int tj = 0; tj < 2; ++tj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gj = j0 + wj * 32 + 16 * tj + lr + 4 * r;
                    if (gj >= n) continue;
                    C[gi + (int64_t)gj * ldc] = alpha * acc[ti][tj][r] + beta * cold[ti][tj][r];
                }
        }
    }
    gsync();
}

// Cholesky of the leading n x n of A (lower triangle used and overwritten).
// Returns 0, or the 1-based index of the first non-positive pivot.
// A of half-bandwidth bw (entries with |r - c| > bw zero): the factor keeps
// the band, so each panel reads only the columns within bw to its left and
// updates only the rows within bw below it.
__device__ __attribute__((noinline)) int wg_potrf(int n, int bw, double* A, int64_t lda, Lds& s) {
    const int t = threadIdx.x;
    gdouble* gA = (gdouble*)A;
    for (int j0 = 0; j0 < n; j0 += PB) {
        const int jb = min(PB, n - j0);
        const int re = min(n, j0 + jb + bw);  // rows of the panel's column block that can be non-zero
        const int kl = max(0, j0 - bw);       // first column that row block j0 can reach
        if (j0 > kl)
            wg_gemm(false, true, re - j0, jb, j0 - kl, -1.0, A + j0 + (int64_t)kl * lda, lda,
                    A + j0 + (int64_t)kl * lda, lda, 1.0, A + j0 + (int64_t)j0 * lda, lda, s);
        for (int e = t; e < jb * jb; e += BT) {
            const int r = e % jb, c = e / jb;
            s.D[r][c] = gA[j0 + r + (int64_t)(j0 + c) * lda];
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
            if (r >= c) gA[j0 + r + (int64_t)(j0 + c) * lda] = s.D[r][c];
        }
        // rows below the block: x L_jj^T = a
        // (the row's jb entries are loaded before the first is used)
        for (int r = j0 + jb + t; r < re; r += BT) {
            keep_lds_reads_here();
            gdouble* ar = gA + r + (int64_t)j0 * lda;
            double x[PB];
#pragma unroll
            for (int c = 0; c < PB; ++c) x[c] = ar[(int64_t)(c < jb ? c : 0) * lda];
#pragma unroll
            for (int c = 0; c < PB; ++c) {
                double v = x[c];
#pragma unroll
                for (int q = 0; q < c; ++q) v -= x[q] * s.D[c][q];
                x[c] = (c < jb) ? v / s.D[c][c] : 0.0;
            }
#pragma unroll
            for (int c = 0; c < PB; ++c)
                if (c < jb) ar[(int64_t)c * lda] = x[c];
        }
        gsync();
    }
    return 0;
}

// Solve L X = B in place (L lower, n x n; B n x nrhs).
// L of half-bandwidth bw: the updates below a block reach only the bw rows
// under it.
__device__ __attribute__((noinline)) void wg_trsm_ln(int n, int bw, int nrhs, const double* L, int64_t ldl, double* B, int64_t ldb, Lds& s) {
    const int t = threadIdx.x;
    const gdouble* gL = (const gdouble*)L;
    gdouble* gB = (gdouble*)B;
    // Two-level blocking: PB-row blocks are solved and update only the rest
    // of their OB-row group (k = PB); each finished group then updates all
    // rows below it in one product with k = OB, so the trailing rows are
    // read and written once per group instead of once per block.
    for (int o0 = 0; o0 < n; o0 += OB) {
        const int oe = min(n, o0 + OB);
        for (int i0 = o0; i0 < oe; i0 += PB) {
            const int ib = min(PB, oe - i0);
            for (int e = t; e < PB * PB; e += BT) {
                const int r = e % PB, c = e / PB;
                s.D[r][c] = (r < ib && c <= r) ? gL[i0 + r + (int64_t)(i0 + c) * ldl] : 0.0;
            }
            __syncthreads();
            // (the column's ib entries are loaded before the first is used)
            for (int j = t; j < nrhs; j += BT) {
                keep_lds_reads_here();
                gdouble* bj = gB + i0 + (int64_t)j * ldb;
                double x[PB];
#pragma unroll
                for (int r = 0; r < PB; ++r) x[r] = bj[r < ib ? r : 0];
#pragma unroll
                for (int r = 0; r < PB; ++r) {
                    double v = x[r];
#pragma unroll
                    for (int q = 0; q < r; ++q) v -= s.D[r][q] * x[q];
                    x[r] = (r < ib) ? v / s.D[r][r] : 0.0;
                }
#pragma unroll
                for (int r = 0; r < PB; ++r)
                    if (r < ib) bj[r] = x[r];
            }
            gsync();
            const int ue = min(oe, i0 + ib + bw);
            if (i0 + ib < ue)
                wg_gemm(false, false, ue - i0 - ib, nrhs, ib, -1.0, L + i0 + ib + (int64_t)i0 * ldl, ldl, B + i0, ldb,
                        1.0, B + i0 + ib, ldb, s);
        }
        const int ge = min(n, oe + bw);
        const int gk = max(o0, oe - bw);  // columns of the group that reach below it
        if (oe < ge)
            wg_gemm(false, false, ge - oe, nrhs, oe - gk, -1.0, L + oe + (int64_t)gk * ldl, ldl, B + gk, ldb, 1.0,
                    B + oe, ldb, s);
    }
}

// Solve L^T X = B in place (two-level blocking as in wg_trsm_ln, from the
// last group up: within a group k = PB, the rows above it get one k = OB
// product).
__device__ __attribute__((noinline)) void wg_trsm_lt(int n, int bw, int nrhs, const double* L, int64_t ldl, double* B, int64_t ldb, Lds& s) {
    const int t = threadIdx.x;
    const gdouble* gL = (const gdouble*)L;
    gdouble* gB = (gdouble*)B;
    const int ngrp = (n + OB - 1) / OB;
    for (int gi = ngrp - 1; gi >= 0; --gi) {
        const int o0 = gi * OB, oe = min(n, o0 + OB);
        const int nblk = (oe - o0 + PB - 1) / PB;
        for (int bi = nblk - 1; bi >= 0; --bi) {
            const int i0 = o0 + bi * PB, ib = min(PB, oe - i0);
            for (int e = t; e < PB * PB; e += BT) {
                const int r = e % PB, c = e / PB;
                s.D[r][c] = (r < ib && c <= r) ? gL[i0 + r + (int64_t)(i0 + c) * ldl] : 0.0;
            }
            __syncthreads();
            // (the column's ib entries are loaded before the first is used;
            // D is zero outside its ib x ib block, so x[q >= ib] = 0 drops out)
            for (int j = t; j < nrhs; j += BT) {
                keep_lds_reads_here();
                gdouble* bj = gB + i0 + (int64_t)j * ldb;
                double x[PB];
#pragma unroll
                for (int r = 0; r < PB; ++r) x[r] = bj[r < ib ? r : 0];
#pragma unroll
                for (int r = PB - 1; r >= 0; --r) {
                    double v = x[r];
#pragma unroll
                    for (int q = r + 1; q < PB; ++q) v -= s.D[q][r] * x[q];
                    x[r] = (r < ib) ? v / s.D[r][r] : 0.0;
                }
#pragma unroll
                for (int r = 0; r < PB; ++r)
                    if (r < ib) bj[r] = x[r];
            }
            gsync();
            const int us = max(o0, i0 - bw);  // rows above the block that it reaches
            if (i0 > us)
                wg_gemm(true, false, i0 - us, nrhs, ib, -1.0, L + i0 + (int64_t)us * ldl, ldl, B + i0, ldb, 1.0,
                        B + us, ldb, s);
        }
        const int gs = max(0, o0 - bw);
        const int gk = min(oe, o0 + bw);  // rows of the group that reach above it
        if (o0 > gs)
            wg_gemm(true, false, o0 - gs, nrhs, gk - o0, -1.0, L + o0 + (int64_t)gs * ldl, ldl, B + o0, ldb, 1.0,
                    B + gs, ldb, s);
    }
}

// In the tridiagonalisation thread t owns the global rows g = t + q BT
// (q < RPT) of A for the whole reduction, so every element of A is read and
// written by one thread only and only LDS carries data between threads.

// Householder reflector of x = A[g0 : g0 + m, c] (x[0] = alpha at row g0):
// x[1:] is scaled in place into v[1:] (also copied to the LDS vector v,
// indexed from row g0).  Returns tau; beta goes to *beta.
template <class Ptr>
__device__ double wg_house(int n, int64_t g0, int m, Ptr col, double alpha, double* v, double* beta, Lds& s) {
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
// The streamed matrix is addressed as global memory (gdouble).

// Rows t + q BT (q < RPT) of columns g0 + j0 .. g0 + j0 + SU - 1.  The loads
// are unconditional within a wave, from a row and column clamped into the
// matrix; entries that are not the caller's (rows it does not own, columns
// j >= m) are never used.  With SKIP, a wave whose rows in slot q all lie
// above the trailing block (rows <= g0) loads nothing there and gets zeros
// (for a caller that only reads the chunk; the unblocked tridiagonalisation
// stores every loaded row back).
template <bool SKIP>
__device__ inline void sytrd_load_chunk(const gdouble* A, int64_t lda, int64_t g0, int j0, int m, int n,
                                        double (&buf)[SU][RPT]) {
    const int t = threadIdx.x;
    const int wlast = __builtin_amdgcn_readfirstlane(t | 63);  // last row of this wave in slot 0
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        if (!SKIP || wlast + q * BT > g0) {
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const int j = (j0 + u < m) ? j0 + u : m - 1;
                const int g = t + q * BT;
                buf[u][q] = A[(g0 + j) * lda + (g < n ? g : n - 1)];
            }
        } else {
#pragma unroll
            for (int u = 0; u < SU; ++u) buf[u][q] = 0.0;
        }
    }
}

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
#pragma unroll 16
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
            // (c) rows/columns g0+1.. : A -= v w^T + w v^T, fused with acc = A v'.
            // Columns are streamed in chunks of SU; the next chunk is loaded
            // before the current one is updated and stored, so each chunk
            // waits for one memory round trip instead of each column.
            const double* v2 = s.va[nxt];  // indexed from global row g0+1
            double acc[RPT], vi[RPT], wi[RPT];
            bool own[RPT];
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int64_t g = t + q * BT, i = g - g0;
                own[q] = g < n && i >= 1;
                vi[q] = own[q] ? v[i] : 0.0;
                wi[q] = own[q] ? w[i] : 0.0;
                acc[q] = 0.0;
            }
            // Two chunk buffers in turn (no copies between them): while one
            // is updated and stored, the loads of the next are in flight.
            // Full chunk pairs run without branches, so that the compiler can
            // count the loads still in flight instead of draining them: rows
            // above the trailing block store their value back unchanged (no
            // other thread touches row g), and a row past the matrix stores
            // row t's final value to row t once more, after row t's store.
            double ca[SU][RPT], cb[SU][RPT];
            const gdouble* gA = (const gdouble*)A;
            gdouble* wA = (gdouble*)A;
            int64_t roff[RPT];
            bool valid[RPT];
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                valid[q] = t + q * BT < n;
                roff[q] = valid[q] ? t + q * BT : t;
            }
            auto process = [&](const double (&cur)[SU][RPT], int j0) {
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    const int j = j0 + u;
                    const double vj = v[j], wj = w[j], v2j = v2[j - 1];
                    gdouble* col = wA + (g0 + j) * lda;
                    double a0 = 0.0;
#pragma unroll
                    for (int q = 0; q < RPT; ++q) {
                        const double p1 = __dmul_rn(vi[q], wj), p2 = __dmul_rn(wi[q], vj);
                        double a = own[q] ? __dsub_rn(cur[u][q], __dadd_rn(p1, p2)) : cur[u][q];
                        if (q == 0) a0 = a;
                        a = valid[q] ? a : a0;
                        col[roff[q]] = a;
                        acc[q] = fma(a, v2j, acc[q]);
                    }
                }
            };
            auto process_tail = [&](const double (&cur)[SU][RPT], int j0) {
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    const int j = j0 + u;
                    if (j < m) {
                        const double vj = v[j], wj = w[j], v2j = v2[j - 1];
                        gdouble* col = wA + (g0 + j) * lda;
#pragma unroll
                        for (int q = 0; q < RPT; ++q) {
                            if (own[q]) {
                                const double p1 = __dmul_rn(vi[q], wj), p2 = __dmul_rn(wi[q], vj);
                                const double a = __dsub_rn(cur[u][q], __dadd_rn(p1, p2));
                                col[t + q * BT] = a;
                                acc[q] = fma(a, v2j, acc[q]);
                            }
                        }
                    }
                }
            };
            if (t < n) {
                sytrd_load_chunk<false>(gA, lda, g0, 1, m, n, ca);
                int j0 = 1;
                // (the first use of a buffer after the loop's back edge waits
                // for every load, so the loop body holds two pairs)
                for (; j0 + 4 * SU <= m; j0 += 4 * SU) {
                    sytrd_load_chunk<false>(gA, lda, g0, j0 + SU, m, n, cb);
                    process(ca, j0);
                    sytrd_load_chunk<false>(gA, lda, g0, j0 + 2 * SU, m, n, ca);
                    process(cb, j0 + SU);
                    sytrd_load_chunk<false>(gA, lda, g0, j0 + 3 * SU, m, n, cb);
                    process(ca, j0 + 2 * SU);
                    sytrd_load_chunk<false>(gA, lda, g0, j0 + 4 * SU, m, n, ca);
                    process(cb, j0 + 3 * SU);
                }
                if (j0 + 2 * SU <= m) {
                    sytrd_load_chunk<false>(gA, lda, g0, j0 + SU, m, n, cb);
                    process(ca, j0);
                    sytrd_load_chunk<false>(gA, lda, g0, j0 + 2 * SU, m, n, ca);
                    process(cb, j0 + SU);
                    j0 += 2 * SU;
                }
                if (j0 < m) {
                    sytrd_load_chunk<false>(gA, lda, g0, j0 + SU, m, n, cb);
                    process_tail(ca, j0);
                    if (j0 + SU < m) process_tail(cb, j0 + SU);
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

// Blocked variant for n >= SYTRD_BLK_MIN: the rank-2 updates of up to NBB
// consecutive steps stay pending in P = [V | W | V] (global, n x 3 NBB,
// ld n, zeros above each vector's first row) and are applied to the
// trailing matrix every NBB steps in one workgroup product with k = 2 NBB,
// [V W] [W V]^T (the column ranges of P that start at 0 and at NBB).  A
// step sees the current matrix through them: its column gets the pending
// updates before the Householder step, and the product with the new v is
// formed from the stale matrix (one read-only pass instead of a read-write
// pass) and corrected by V (W^T v) + W (V^T v).  Same reflectors as
// wg_sytrd in exact arithmetic.
constexpr int NBB = 32;
constexpr int SYTRD_BLK_MIN = 256;
constexpr int PU = 8;  // pending pairs read per batch of loads

// Entries of pending pairs i0 .. i0+PU-1 (clamped to np-1) at this thread's
// rows (clamped to n-1): all loads issued before any is used, so a batch
// costs one memory latency instead of PU.
__device__ inline void pend_rows(const gdouble* PV, const gdouble* PW, int n, int np, int i0,
                                 double (&pv)[PU][RPT], double (&pw)[PU][RPT]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int u = 0; u < PU; ++u) {
        const int64_t i = (i0 + u < np) ? i0 + u : np - 1;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int g = t + q * BT;
            const int64_t gg = g < n ? g : n - 1;
            pv[u][q] = PV[gg + i * n];
            pw[u][q] = PW[gg + i * n];
        }
    }
}

__device__ __attribute__((noinline)) void wg_sytrd_blk(int n, double* Ag, int64_t lda, double* taug, double* P, Lds& s) {
    const int t = threadIdx.x;
    gdouble* A = (gdouble*)Ag;
    gdouble* tau = (gdouble*)taug;
    gdouble* PV = (gdouble*)P;           // column i: v_i (global rows)
    gdouble* PW = PV + (int64_t)NBB * n; // column i: w_i
    int np = 0;                        // pending pairs
    // append (v, w) of the reflector whose first row is r1 (v, w indexed from r1)
    auto append = [&](int r1, const double* v, const double* w) {
        for (int g = t; g < n; g += BT) {
            const bool in = g >= r1;
            const double vg = in ? v[g - r1] : 0.0;
            PV[g + (int64_t)np * n] = vg;
            PW[g + (int64_t)np * n] = in ? w[g - r1] : 0.0;
            PW[g + (int64_t)(NBB + np) * n] = vg;
        }
        ++np;
        gsync();
    };
    // A[f:, f:] -= V W^T + W V^T over the pending pairs
    auto flush = [&](int f) {
        if (np > 0 && f < n) {
            const int mm = n - f;
            double* pv = P + f;
            double* pw = P + (int64_t)NBB * n + f;
            double* a = Ag + f + (int64_t)f * lda;
            if (np == NBB) {
                wg_gemm(false, true, mm, mm, 2 * NBB, -1.0, pv, n, pw, n, 1.0, a, lda, s);
            } else {
                wg_gemm(false, true, mm, mm, np, -1.0, pv, n, pw, n, 1.0, a, lda, s);
                wg_gemm(false, true, mm, mm, np, -1.0, pw, n, pv, n, 1.0, a, lda, s);
            }
        }
        np = 0;
    };
    // reflector 0 and w_0 (no pending updates yet)
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
            const gdouble* col = A + (int64_t)j * lda;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int g = t + q * BT;
                if (g >= 1 && g < n) acc[q] = fma(col[g], vj, acc[q]);
            }
        }
        wg_make_w(n, 1, n - 1, tk, acc, s.va[0], s.wa[0], s);
        append(1, s.va[0], s.wa[0]);
    }
    const gdouble* gA = A;
    for (int k = 0; k < n - 3; ++k) {
        const int nxt = (k + 1) & 1;
        const int64_t g0 = k + 1;  // column of reflector k+1, first row/column of A22
        const int m = n - k - 1;   // order of A22
        if (np == NBB) flush((int)g0);
        // (a) column g0, rows g0.., with the pending updates (row g0 of the
        // pending pairs staged in LDS first)
        {
            double* r0 = &s.qx[1][0];  // [0, NBB): v_i[g0], [NBB, 2 NBB): w_i[g0]
            if (t < np) {
                r0[t] = PV[g0 + (int64_t)t * n];
                r0[NBB + t] = PW[g0 + (int64_t)t * n];
            }
            __syncthreads();
            gdouble* c0 = A + g0 * lda;
            double a[RPT];
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int g = t + q * BT;
                a[q] = c0[g < n ? g : n - 1];
            }
            for (int i0 = 0; i0 < np; i0 += PU) {
                double pv[PU][RPT], pw[PU][RPT];
                pend_rows(PV, PW, n, np, i0, pv, pw);
#pragma unroll
                for (int u = 0; u < PU; ++u) {
                    if (i0 + u < np) {
#pragma unroll
                        for (int q = 0; q < RPT; ++q)
                            a[q] -= pv[u][q] * r0[NBB + i0 + u] + pw[u][q] * r0[i0 + u];
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int64_t g = t + q * BT;
                if (g < n && g >= g0) {
                    c0[g] = a[q];
                    if (g == g0) s.dval[0] = a[q];
                    if (g == g0 + 1) s.dval[1] = a[q];
                }
            }
        }
        gsync();
        // (b) reflector k+1 from rows g0+1.. of that column
        double beta;
        const double tk = wg_house(n, g0 + 1, m - 1, A + g0 * lda, s.dval[1], s.va[nxt], &beta, s);
        if (t == 0) {
            s.dd[k + 1] = s.dval[0];
            s.ee[k + 1] = beta;
            tau[k + 1] = tk;
        }
        __syncthreads();
        const double* v2 = s.va[nxt];  // indexed from global row g0+1
        // (c) acc = A22_stale v2: one read-only pass, two chunk buffers in turn
        double acc[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) acc[q] = 0.0;
        if (t < n) {
            double ca[SU][RPT], cb[SU][RPT];
            auto mac = [&](const double (&cur)[SU][RPT], int j0) {
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    const int j = j0 + u;
                    const double v2j = (j < m) ? v2[j - 1] : 0.0;
#pragma unroll
                    for (int q = 0; q < RPT; ++q) acc[q] = fma(cur[u][q], v2j, acc[q]);
                }
            };
            sytrd_load_chunk<true>(gA, lda, g0, 1, m, n, ca);
            int j0 = 1;
            for (; j0 + 2 * SU <= m; j0 += 2 * SU) {
                sytrd_load_chunk<true>(gA, lda, g0, j0 + SU, m, n, cb);
                mac(ca, j0);
                sytrd_load_chunk<true>(gA, lda, g0, j0 + 2 * SU, m, n, ca);
                mac(cb, j0 + SU);
            }
            if (j0 < m) {
                sytrd_load_chunk<true>(gA, lda, g0, j0 + SU, m, n, cb);
                mac(ca, j0);
                mac(cb, j0 + SU);
            }
        }
        // corrections: acc -= V (W^T v2) + W (V^T v2) over rows g0+1..
        {
            double* dots = &s.qx[0][0];  // 2 NBB sums: alpha_i = w_i^T v2, beta_i = v_i^T v2
            double vg[RPT];
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int64_t g = t + q * BT;
                vg[q] = (g < n && g >= g0 + 1) ? v2[g - g0 - 1] : 0.0;
            }
            for (int i0 = 0; i0 < np; i0 += PU) {
                double pv[PU][RPT], pw[PU][RPT];
                pend_rows(PV, PW, n, np, i0, pv, pw);
#pragma unroll
                for (int u = 0; u < PU; ++u) {
                    if (i0 + u < np) {
                        double pa = 0.0, pb = 0.0;
#pragma unroll
                        for (int q = 0; q < RPT; ++q) {
                            pa += pw[u][q] * vg[q];
                            pb += pv[u][q] * vg[q];
                        }
                        for (int o = 32; o > 0; o >>= 1) {
                            pa += __shfl_xor(pa, o, 64);
                            pb += __shfl_xor(pb, o, 64);
                        }
                        if ((t & 63) == 0) {
                            s.qy[0][(t >> 6) * 2 * NBB + i0 + u] = pa;
                            s.qy[0][(t >> 6) * 2 * NBB + NBB + i0 + u] = pb;
                        }
                    }
                }
            }
            __syncthreads();
            if (t < 2 * np) {
                const int i = (t < np) ? t : NBB + (t - np);
                double a = 0.0;
                for (int w = 0; w < BT / 64; ++w) a += s.qy[0][w * 2 * NBB + i];
                dots[i] = a;
            }
            __syncthreads();
            double c[RPT];
#pragma unroll
            for (int q = 0; q < RPT; ++q) c[q] = 0.0;
            for (int i0 = 0; i0 < np; i0 += PU) {
                double pv[PU][RPT], pw[PU][RPT];
                pend_rows(PV, PW, n, np, i0, pv, pw);
#pragma unroll
                for (int u = 0; u < PU; ++u) {
                    if (i0 + u < np) {
#pragma unroll
                        for (int q = 0; q < RPT; ++q) c[q] += pv[u][q] * dots[i0 + u] + pw[u][q] * dots[NBB + i0 + u];
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int64_t g = t + q * BT;
                if (g < n && g >= g0 + 1) acc[q] -= c[q];
            }
        }
        // (d) w of step k+1, then the pair joins the pending ones
        wg_make_w(n, g0 + 1, m - 1, tk, acc, v2, s.wa[nxt], s);
        append((int)g0 + 1, v2, s.wa[nxt]);
    }
    // the last 2 x 2 block, rows and columns n-2, n-1, after all pending updates
    flush(n - 2);
    gsync();
    if (t == 0) {
        s.dd[n - 2] = A[(n - 2) + (int64_t)(n - 2) * lda];
        s.ee[n - 2] = A[(n - 1) + (int64_t)(n - 2) * lda];
        s.dd[n - 1] = A[(n - 1) + (int64_t)(n - 1) * lda];
        s.ee[n - 1] = 0.0;
    }
    __syncthreads();
}

// Z := Q Z with Q = H_0 H_1 ... H_{n-3} from wg_sytrd, applied as block
// reflectors of PB consecutive H (forward, columnwise: I - V T V^T), last
// block first.  work: >= 3 PB n + PB PB doubles.
// Work of wg_ormtr with block width w, and the size of its work array.
__host__ __device__ inline int64_t ormtr_need(int64_t n, int64_t w) {
    return (n - 1) * w + 2 * w * w + w * PB + 2 * w * n;
}
__host__ __device__ inline int64_t ormtr_wsz(int64_t n) {
    return n * n > ormtr_need(n, PB) ? n * n : ormtr_need(n, PB);
}

__device__ __attribute__((noinline)) void wg_ormtr(int n, const double* A, int64_t lda, const double* tau, double* Z, int64_t ldz,
                         double* work, Lds& s) {
    const int t = threadIdx.x;
    const int nref = n - 2;
    if (nref <= 0) return;
    const gdouble* gA = (const gdouble*)A;
    const gdouble* gtau = (const gdouble*)tau;
    // Block reflectors of QW = 4 PB reflectors when the n x n work array has
    // room (one pass over Z per 128 reflectors instead of per 32), else PB.
    // T of a wide block: its PB x PB diagonal blocks by the column recurrence
    // in LDS, the blocks above them from T(0:c0, S) = -T(0:c0, 0:c0)
    // G(0:c0, S) T_SS with G = V^T V.
    constexpr int QW = 4 * PB;
    const int W = (ormtr_need(n, QW) <= ormtr_wsz(n)) ? QW : PB;
    const int nblk = (nref + W - 1) / W;
    for (int bi = nblk - 1; bi >= 0; --bi) {
        const int k0 = bi * W, nb = min(W, nref - k0);
        const int rows = n - k0 - 1;  // rows k0+1 .. n-1
        double* Vb = work;                          // rows x nb
        gdouble* gV = (gdouble*)Vb;
        double* Tm = Vb + (int64_t)rows * W;        // W x W
        double* Gm = Tm + W * W;                    // W x W
        double* Xm = Gm + W * W;                    // W x PB
        double* Wt = Xm + W * PB;                   // nb x n
        double* Wt2 = Wt + (int64_t)W * n;          // nb x n
        // V of the block, eight columns' loads in flight before their stores
        for (int c0 = 0; c0 < nb; c0 += 8)
            for (int rr = t; rr < rows; rr += BT) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int c = min(c0 + u, nb - 1);
                    v[u] = gA[(k0 + 1 + rr) + (int64_t)(k0 + c) * lda];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int c = c0 + u;
                    if (c < nb) gV[rr + (int64_t)c * rows] = rr < c ? 0.0 : (rr == c ? 1.0 : v[u]);
                }
            }
        for (int e = t; e < W * W; e += BT) ((gdouble*)Tm)[e] = 0.0;
        gsync();
        wg_gemm(true, false, nb, nb, rows, 1.0, Vb, rows, Vb, rows, 0.0, Gm, W, s);
        for (int c0 = 0; c0 < nb; c0 += PB) {
            const int sb = min(PB, nb - c0);
            // T_SS: T[c][c] = tau_c, T[0:c, c] = -tau_c T[0:c, 0:c] G[0:c, c] (within the sub-block)
            for (int e = t; e < PB * PB; e += BT) s.D[e % PB][e / PB] = 0.0;
            __syncthreads();
            for (int c = 0; c < sb; ++c) {
                const double tc = gtau[k0 + c0 + c];
                double acc = 0.0;
                if (t < c) {
                    for (int q = t; q < c; ++q) acc += s.D[t][q] * ((const gdouble*)Gm)[(c0 + q) + (int64_t)(c0 + c) * W];
                }
                __syncthreads();
                if (t < c) s.D[t][c] = -tc * acc;
                if (t == c) s.D[c][c] = tc;
                __syncthreads();
            }
            for (int e = t; e < PB * PB; e += BT) {
                const int r = e % PB, c = e / PB;
                if (r < sb && c < sb) ((gdouble*)Tm)[(c0 + r) + (int64_t)(c0 + c) * W] = s.D[r][c];
            }
            gsync();
            if (c0 > 0) {
                // T(0:c0, S) = -(T(0:c0, 0:c0) G(0:c0, S)) T_SS
                wg_gemm(false, false, c0, sb, c0, 1.0, Tm, W, Gm + (int64_t)c0 * W, W, 0.0, Xm, W, s);
                wg_gemm(false, false, c0, sb, sb, -1.0, Xm, W, Tm + c0 + (int64_t)c0 * W, W, 0.0,
                        Tm + (int64_t)c0 * W, W, s);
            }
        }
        wg_gemm(true, false, nb, n, rows, 1.0, Vb, rows, Z + k0 + 1, ldz, 0.0, Wt, nb, s);
        wg_gemm(false, false, nb, n, nb, 1.0, Tm, W, Wt, nb, 0.0, Wt2, nb, s);
        wg_gemm(false, false, rows, n, nb, -1.0, Vb, rows, Wt2, nb, 1.0, Z + k0 + 1, ldz, s);
    }
}

// ---------------------------------------------------------------------------
// Tridiagonal eigensolver: Cuppen's divide and conquer inside one workgroup.
//
// T = diag(T1, T2) + |beta| u u^T, u = e_s + sign(beta) e_{s+1} (beta the
// coupling entry at the split s; the last diagonal entry of T1 and the first
// of T2 are reduced by |beta|).  With T1 = Q1 D1 Q1^T, T2 = Q2 D2 Q2^T the
// merged problem is D + rho z z^T, z = Q^T u / sqrt 2, rho = 2 |beta|.  Poles
// with rho |z_j| <= tol, or made to share one z by a Givens rotation whose
// residue is <= tol, deflate; each remaining root is found by one thread in
// coordinates shifted to its nearer pole; z is recomputed from the roots
// (Gu and Eisenstat) and the merged vectors are Q times the normalised
// columns zhat / (d - lambda_k), with Q's block structure (columns living in
// one half only) used by the two GEMMs.  Leaves (<= DCL) use implicit QL,
// one wave per leaf, in LDS.

__device__ inline void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS tile of wave w: va[0..1], wa[0..1] (contiguous) for w < 4, qx, qy for w >= 4.
__device__ inline double* dc_tile(Lds& s, int w) {
    static_assert(sizeof(s.va) + sizeof(s.wa) == 4 * NMAX * sizeof(double), "va, wa contiguous");
    return w < 4 ? &s.va[0][0] + w * NMAX : &s.qx[0][0] + (w - 4) * NMAX;
}

// Leaves: wave w solves leaves w, w + 8, ...  Returns 0 or 1 (QL failed).
__device__ __attribute__((noinline)) int dc_leaves(int nleaf, double* Z, int64_t ldz, Lds& s) {
    static_assert(BT / 64 == 8 && DCL * DCL <= NMAX, "eight leaf tiles of DCL x DCL in LDS");
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    double* zt = dc_tile(s, w);
    double* ld = s.lq[w][0];
    double* le = s.lq[w][1];
    double* rc = s.lq[w][2];
    double* rs = s.lq[w][3];
    int failed = 0;
    for (int li = w; li < nleaf; li += BT / 64) {
        const int lo = s.lb[li], m = s.lb[li + 1] - lo;
        if (lane < m) {
            for (int c = 0; c < m; ++c) zt[lane + DCL * c] = (lane == c) ? 1.0 : 0.0;
            ld[lane] = s.dd[lo + lane];
            le[lane] = (lane < m - 1) ? s.ee[lo + lane] : 0.0;
        }
        wsync();
        for (int l = 0; l < m && !failed; ++l) {
            int iter = 0;
            for (;;) {
                int go = 0, rlo = 0, rhi = -1;
                if (lane == 0) {
                    int mm = l;
                    while (mm < m - 1) {
                        if (fabs(le[mm]) <= EPS * (fabs(ld[mm]) + fabs(ld[mm + 1]))) break;
                        ++mm;
                    }
                    if (mm != l) {
                        if (++iter > 90) {
                            go = -1;
                        } else {
                            go = 1;
                            double g = (ld[l + 1] - ld[l]) / (2.0 * le[l]);
                            double r = hypot(g, 1.0);
                            g = ld[mm] - ld[l] + le[l] / (g + (g >= 0.0 ? r : -r));
                            double sn = 1.0, c = 1.0, p = 0.0;
                            int i = mm - 1;
                            bool early = false;
                            for (; i >= l; --i) {
                                const double f = sn * le[i], b = c * le[i];
                                r = hypot(f, g);
                                le[i + 1] = r;
                                if (r == 0.0) {
                                    ld[i + 1] -= p;
                                    le[mm] = 0.0;
                                    early = true;
                                    break;
                                }
                                sn = f / r;
                                c = g / r;
                                g = ld[i + 1] - p;
                                r = (ld[i] - g) * sn + 2.0 * c * b;
                                p = sn * r;
                                ld[i + 1] = g + p;
                                g = c * r - b;
                                rc[i] = c;
                                rs[i] = sn;
                            }
                            rlo = early ? i + 1 : l;
                            rhi = mm - 1;
                            if (!early) {
                                ld[l] -= p;
                                le[l] = g;
                                le[mm] = 0.0;
                            }
                        }
                    }
                }
                go = __shfl(go, 0, 64);
                rlo = __shfl(rlo, 0, 64);
                rhi = __shfl(rhi, 0, 64);
                wsync();
                if (go < 0) failed = 1;
                if (go <= 0) break;
                if (lane < m) {
                    for (int i = rhi; i >= rlo; --i) {
                        const double c = rc[i], sn = rs[i];
                        const double f = zt[lane + (i + 1) * DCL], a = zt[lane + i * DCL];
                        zt[lane + (i + 1) * DCL] = sn * a + c * f;
                        zt[lane + i * DCL] = c * a - sn * f;
                    }
                }
                wsync();
            }
        }
        if (lane < m) {
            s.dd[lo + lane] = ld[lane];
            for (int c = 0; c < m; ++c) Z[(lo + lane) + (int64_t)(lo + c) * ldz] = zt[lane + DCL * c];
        }
        wsync();
    }
    return failed;
}

// WG-wide max of v >= 0.
__device__ double wg_max(double v, Lds& s) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s.red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < BT / 64; ++w) r = fmax(r, s.red[w]);
    __syncthreads();
    return r;
}

// Secular equation root k of 1 + rho sum_j z_j^2 / (d_j - lambda) = 0 (d
// ascending, K poles): returns tau with lambda = d[org] + tau; false if the
// iteration did not converge.
__device__ bool dc_root(int K, int k, const double* d, const double* z, double rho, int* org_out, double* tau_out) {
    int org;
    double lo, hi;
    if (k < K - 1) {
        const double mid = 0.5 * (d[k + 1] - d[k]);
        double f = 1.0;
        for (int j = 0; j < K; ++j) f += rho * z[j] * z[j] / ((d[j] - d[k]) - mid);
        if (f >= 0.0) {
            org = k;
            lo = 0.0;
            hi = mid;
        } else {
            org = k + 1;
            lo = -mid;
            hi = 0.0;
        }
    } else {
        org = k;
        double zz = 0.0;
        for (int j = 0; j < K; ++j) zz += z[j] * z[j];
        lo = 0.0;
        hi = rho * zz;
    }
    const double dorg = d[org];
    const double Dk = d[k] - dorg;
    const double Dk1 = (k < K - 1) ? d[k + 1] - dorg : 0.0;
    double x = 0.5 * (lo + hi);
    bool conv = false;
    for (int it = 0; it < 400; ++it) {
        double psi = 0.0, phi = 0.0, dpsi = 0.0, dphi = 0.0;
        for (int j = 0; j <= k; ++j) {
            const double dl = (d[j] - dorg) - x;
            const double tq = rho * z[j] * z[j] / dl;
            psi += tq;
            dpsi += tq / dl;
        }
        for (int j = k + 1; j < K; ++j) {
            const double dl = (d[j] - dorg) - x;
            const double tq = rho * z[j] * z[j] / dl;
            phi += tq;
            dphi += tq / dl;
        }
        const double f = 1.0 + psi + phi;
        if (f < 0.0)
            lo = x;
        else
            hi = x;
        if (fabs(f) <= 8.0 * EPS * (1.0 + fabs(psi) + fabs(phi)) || hi - lo <= 2.0 * EPS * fmax(fabs(lo), fabs(hi))) {
            conv = true;
            break;
        }
        // two-pole rational model through f, f' (poles d_k, d_k+1), safeguarded by the bracket
        const double dlk = Dk - x;
        const double bb = dpsi * dlk * dlk;
        double a2, a1, a0;
        if (k < K - 1) {
            const double dlk1 = Dk1 - x;
            const double BB = dphi * dlk1 * dlk1;
            const double c = f - dpsi * dlk - dphi * dlk1;
            a2 = c;
            a1 = -(c * (Dk + Dk1) + bb + BB);
            a0 = c * Dk * Dk1 + bb * Dk1 + BB * Dk;
        } else {
            const double c = f - dpsi * dlk;
            a2 = 0.0;
            a1 = -c;
            a0 = c * Dk + bb;
        }
        double xn = 0.5 * (lo + hi);
        if (a2 == 0.0) {
            if (a1 != 0.0) {
                const double cnd = -a0 / a1;
                if (cnd > lo && cnd < hi) xn = cnd;
            }
        } else {
            const double disc = a1 * a1 - 4.0 * a2 * a0;
            if (disc >= 0.0) {
                const double sq = sqrt(disc);
                const double q = -0.5 * (a1 + (a1 >= 0.0 ? sq : -sq));
                const double c1 = q / a2;
                const double c2 = (q != 0.0) ? a0 / q : c1;
                if (c1 > lo && c1 < hi)
                    xn = c1;
                else if (c2 > lo && c2 < hi)
                    xn = c2;
            }
        }
        x = xn;
    }
    *org_out = org;
    *tau_out = x;
    return conv;
}

// Merge of the blocks [o, o+n1) and [o+n1, o+N) (eigenpairs in s.dd and the
// diagonal blocks of Z).  X (N x N), U (K x K), Y (N x K): global work, R:
// rotations (4 N doubles).  Returns 0 or 2 (a root did not converge).
__device__ __attribute__((noinline)) int dc_merge(int o, int N, int n1, double* Z, int64_t ldz, double* X, double* U,
                                                  double* Y, double* R, Lds& s) {
    const int t = threadIdx.x;
    double* ds = s.va[0];   // sorted poles, then the root offsets tau
    double* zs = s.va[1];   // sorted z, then zhat
    double* dk = s.wa[0];   // kept poles
    double* zk = s.wa[1];   // their z
    double* dvl = s.qx[0];  // deflated values
    double* aux = s.qx[1];  // 1 / column norms of U, then the merged values
    int* perm = reinterpret_cast<int*>(s.qy[0]);  // sorted -> child column, then ranks
    int* typ = perm + NMAX;                        // 1 top only, 2 both, 3 bottom only
    int* kcol = reinterpret_cast<int*>(s.qy[1]);   // kept columns
    int* tpos = kcol + NMAX;                       // position of kept column k in type order
    int* rorg = s.rk;                              // pole each root is measured from
    int* dcol = s.ix;                              // deflated columns
    gdouble* gZ = (gdouble*)Z;
    gdouble* gX = (gdouble*)X;
    gdouble* gR = (gdouble*)R;
    gint* ra = (gint*)(gR + 2 * N);
    gint* rb = ra + N;
    gdouble* rcs = gR;
    gdouble* rsn = gR + N;
    const double beta = s.ee[o + n1 - 1];
    const double sgn = beta >= 0.0 ? 1.0 : -1.0;
    const double rho = 2.0 * fabs(beta);
    const double isq2 = 0.70710678118654752440;
    // (a) z from the last row of Q1 and the first row of Q2; sort the poles
    double mx = 0.0;
    for (int i = t; i < N; i += BT) {
        const double vi = s.dd[o + i];
        int r = 0;
        for (int j = 0; j < N; ++j) {
            const double vj = s.dd[o + j];
            r += (vj < vi || (vj == vi && j < i)) ? 1 : 0;
        }
        const double zi = (i < n1 ? gZ[(o + n1 - 1) + (int64_t)(o + i) * ldz] : sgn * gZ[(o + n1) + (int64_t)(o + i) * ldz]) * isq2;
        ds[r] = vi;
        zs[r] = zi;
        perm[r] = i;
        typ[i] = i < n1 ? 1 : 3;
        mx = fmax(mx, fmax(fabs(vi), rho * fabs(zi)));
    }
    const double tol = 8.0 * EPS * wg_max(mx, s);
    // (b) deflation scan (one thread)
    if (t == 0) {
        int K = 0, nd = 0, nr = 0, cand = -1, ccol = -1;
        double cd = 0.0, cz = 0.0;
        for (int q = 0; q < N; ++q) {
            const double dj = ds[q], zj = zs[q];
            const int col = perm[q];
            if (rho * fabs(zj) <= tol) {
                dvl[nd] = dj;
                dcol[nd] = col;
                ++nd;
                continue;
            }
            if (cand < 0) {
                cand = q;
                ccol = col;
                cd = dj;
                cz = zj;
                continue;
            }
            const double r = hypot(cz, zj);
            const double c = zj / r, sn = cz / r;
            if (fabs((dj - cd) * c * sn) <= tol) {
                // rotate columns (ccol, col): the candidate deflates, the new pole carries z = r
                ra[nr] = ccol;
                rb[nr] = col;
                rcs[nr] = c;
                rsn[nr] = sn;
                ++nr;
                if (typ[ccol] != typ[col]) {
                    typ[ccol] = 2;
                    typ[col] = 2;
                }
                dvl[nd] = c * c * cd + sn * sn * dj;
                dcol[nd] = ccol;
                ++nd;
                cand = q;
                ccol = col;
                cd = sn * sn * cd + c * c * dj;
                cz = r;
            } else {
                dk[K] = cd;
                zk[K] = cz;
                kcol[K] = ccol;
                ++K;
                cand = q;
                ccol = col;
                cd = dj;
                cz = zj;
            }
        }
        if (cand >= 0) {
            dk[K] = cd;
            zk[K] = cz;
            kcol[K] = ccol;
            ++K;
        }
        int c1 = 0, c2 = 0, c3 = 0;
        for (int k = 0; k < K; ++k) {
            const int ty = typ[kcol[k]];
            c1 += ty == 1;
            c2 += ty == 2;
            c3 += ty == 3;
        }
        int p1 = 0, p2 = c1, p3 = c1 + c2;
        for (int k = 0; k < K; ++k) {
            const int ty = typ[kcol[k]];
            tpos[k] = (ty == 1) ? p1++ : (ty == 2) ? p2++ : p3++;
        }
        s.ival[1] = K;
        s.ival[2] = nr;
        s.qlo[0] = c1;
        s.qlo[1] = c2;
        s.qlo[2] = c3;
        s.ival[3] = 0;
    }
    gsync();
    const int K = s.ival[1], nr = s.ival[2];
    const int c1 = s.qlo[0], c2 = s.qlo[1], c3 = s.qlo[2];
    // (c) deflation rotations on the columns of the merged block, one row per thread
    if (nr > 0) {
        for (int r = t; r < N; r += BT) {
            gdouble* zr = gZ + (o + r);
            for (int q = 0; q < nr; ++q) {
                const int64_t a = o + ra[q], b = o + rb[q];
                const double c = rcs[q], sn = rsn[q];
                const double x = zr[a * ldz], y = zr[b * ldz];
                zr[a * ldz] = c * x - sn * y;
                zr[b * ldz] = sn * x + c * y;
            }
        }
    }
    // (d) roots, one thread each: tau into ds, origin into rorg
    for (int k = t; k < K; k += BT) {
        int org;
        double tau;
        if (!dc_root(K, k, dk, zk, rho, &org, &tau)) s.ival[3] = 2;
        rorg[k] = org;
        ds[k] = tau;
    }
    __syncthreads();
    // (e) zhat_j from the roots (factors paired so that each lies in (0, 1])
    for (int j = t; j < K; j += BT) {
        const double dj = dk[j];
        double p = (ds[K - 1] - (dj - dk[rorg[K - 1]])) / rho;
        for (int k = 0; k < j; ++k) p *= (ds[k] - (dj - dk[rorg[k]])) / (dk[k] - dj);
        for (int k = j; k < K - 1; ++k) p *= (ds[k] - (dj - dk[rorg[k]])) / (dk[k + 1] - dj);
        zs[j] = copysign(sqrt(fabs(p)), zk[j]);
    }
    __syncthreads();
    // (f) U: column k = zhat / (d - lambda_k), normalised; rows in type order
    for (int k = t; k < K; k += BT) {
        const double dorg = dk[rorg[k]], tau = ds[k];
        double ss = 0.0;
        for (int j = 0; j < K; ++j) {
            const double u = zs[j] / ((dk[j] - dorg) - tau);
            ss += u * u;
        }
        aux[k] = 1.0 / sqrt(ss);
    }
    __syncthreads();
    for (int j = t; j < K; j += BT) {
        const double zj = zs[j], dj = dk[j];
        gdouble* ur = (gdouble*)U + tpos[j];
        for (int k = 0; k < K; ++k) ur[(int64_t)k * K] = zj / ((dj - dk[rorg[k]]) - ds[k]) * aux[k];
    }
    // (g) kept columns of Q in type order, deflated columns after them
    // (column k < K of the gathered order is kept column tpos[k], column
    // k >= K deflated column k - K); MV columns loaded before any is stored
    constexpr int MV = 8;
    for (int r = t; r < N; r += BT) {
        const gdouble* zr = gZ + (o + r);
        for (int k0 = 0; k0 < N; k0 += MV) {
            double v[MV];
#pragma unroll
            for (int u = 0; u < MV; ++u) {
                const int k = min(k0 + u, N - 1);
                v[u] = zr[(int64_t)(o + (k < K ? kcol[k] : dcol[k - K])) * ldz];
            }
#pragma unroll
            for (int u = 0; u < MV; ++u) {
                const int k = k0 + u;
                if (k < N) gX[r + (int64_t)(k < K ? tpos[k] : k) * N] = v[u];
            }
        }
    }
    gsync();
    // (h) Y = Q U, top rows from the type 1|2 columns, bottom rows from type 2|3
    if (K > 0) {
        wg_gemm(false, false, n1, K, c1 + c2, 1.0, X, N, U, K, 0.0, Y, N, s);
        wg_gemm(false, false, N - n1, K, c2 + c3, 1.0, X + n1 + (int64_t)c1 * N, N, U + c1, K, 0.0, Y + n1, N, s);
    }
    // (i) merged values (roots, then deflated poles) and their ranks
    for (int c = t; c < N; c += BT) aux[c] = c < K ? dk[rorg[c]] + ds[c] : dvl[c - K];
    __syncthreads();
    for (int c = t; c < N; c += BT) {
        const double vc = aux[c];
        int r = 0;
        for (int j = 0; j < N; ++j) {
            const double vj = aux[j];
            r += (vj < vc || (vj == vc && j < c)) ? 1 : 0;
        }
        perm[c] = r;
    }
    __syncthreads();
    // (j) scatter into Z and s.dd in ascending order
    for (int c0 = 0; c0 < N; c0 += MV) {
        for (int r = t; r < N; r += BT) {
            double v[MV];
#pragma unroll
            for (int u = 0; u < MV; ++u) {
                const int c = min(c0 + u, N - 1);
                v[u] = ((c < K) ? (const gdouble*)Y : (const gdouble*)gX)[r + (int64_t)c * N];
            }
#pragma unroll
            for (int u = 0; u < MV; ++u) {
                const int c = c0 + u;
                if (c < N) gZ[(o + r) + (int64_t)(o + perm[c]) * ldz] = v[u];
            }
        }
    }
    for (int c = t; c < N; c += BT) s.dd[o + perm[c]] = aux[c];
    gsync();
    return s.ival[3];
}

// Eigen-decomposition of the tridiagonal (s.dd, s.ee[0..n-2]) of order n:
// s.dd := eigenvalues (ascending when n > DCL), Z := eigenvectors.  X, U, Y
// (n x n) and R (4 n) are global work.  Returns 0, 1 (a leaf's QL did not
// converge) or 2 (a secular equation did not converge).
__device__ __attribute__((noinline)) int wg_stedc(int n, double* Z, int64_t ldz, double* X, double* U, double* Y,
                                                  double* R, Lds& s) {
    const int t = threadIdx.x;
    // leaves: halve every block until it has at most DCL rows
    int depth = 0;
    while (((n + (1 << depth) - 1) >> depth) > DCL) ++depth;
    const int nleaf = 1 << depth;
    if (t == 0) {
        s.lb[0] = 0;
        s.lb[nleaf] = n;
        for (int d = 0; d < depth; ++d) {
            const int step = nleaf >> d;  // boundaries at depth d are lb[i * step]
            for (int i = 0; i < (1 << d); ++i) {
                const int lo = s.lb[i * step], hi = s.lb[(i + 1) * step];
                s.lb[i * step + step / 2] = lo + (hi - lo) / 2;
            }
        }
        // split adjustment at every boundary
        for (int i = 1; i < nleaf; ++i) {
            const int sp = s.lb[i] - 1;
            const double a = fabs(s.ee[sp]);
            s.dd[sp] -= a;
            s.dd[sp + 1] -= a;
        }
    }
    for (int j = 0; j < n; ++j)
        for (int i = t; i < n; i += BT) Z[i + (int64_t)j * ldz] = 0.0;
    gsync();
    const int lf = dc_leaves(nleaf, Z, ldz, s);
    __syncthreads();
    if (t == 0) s.ival[2] = 0;
    __syncthreads();
    if (lf) s.ival[2] = 1;
    gsync();
    if (s.ival[2]) return 1;
    for (int d = depth - 1; d >= 0; --d) {
        const int step = nleaf >> d;
        for (int i = 0; i < (1 << d); ++i) {
            const int o = s.lb[i * step], N = s.lb[(i + 1) * step] - o, n1 = s.lb[i * step + step / 2] - o;
            const int rc = dc_merge(o, N, n1, Z, ldz, X, U, Y, R, s);
            if (rc) return rc;
        }
    }
    return 0;
}

// f(i, j, src[i + j ls]) for the n x n source (strict: below the diagonal
// only), the loads of MVC columns issued before their values are handed on,
// so a copy costs one memory latency per MVC columns, not per column.
constexpr int MVC = 8;
template <class F>
__device__ inline void wg_cols(int n, bool strict, const double* srcg, int64_t ls, F f) {
    const gdouble* src = (const gdouble*)srcg;
    const int t = threadIdx.x;
    for (int j0 = 0; j0 < n; j0 += MVC) {
        for (int i = (strict ? j0 + 1 : 0) + t; i < n; i += BT) {
            double v[MVC];
#pragma unroll
            for (int u = 0; u < MVC; ++u) v[u] = src[i + (int64_t)min(j0 + u, n - 1) * ls];
#pragma unroll
            for (int u = 0; u < MVC; ++u) {
                const int j = j0 + u;
                if (j < n && (!strict || i > j)) f(i, j, v[u]);
            }
        }
    }
}

__device__ int64_t solve_one(const BProb& p, Lds& s) {
    const int t = threadIdx.x;
    const int n = (int)p.n;
    const int64_t ld = p.ld;
    double *L = p.L, *W = p.W, *A = p.A, *Z = p.Z;
    gdouble *gL = (gdouble*)L, *gW = (gdouble*)W, *gA = (gdouble*)A;
    wg_cols(n, false, p.M, ld, [&](int i, int j, double v) { gL[i + (int64_t)j * n] = v; });
    wg_cols(n, false, p.K, ld, [&](int i, int j, double v) { gW[i + (int64_t)j * n] = v; });
    gsync();
    const int bw = (int)min(p.bw, p.n - 1);
    const int piv = wg_potrf(n, bw, L, n, s);
    if (piv) return piv;
    wg_trsm_ln(n, bw, n, L, n, W, n, s);  // W = L^-1 K
    // A = W^T (reads along columns, so they coalesce; the strided side is
    // the stores, which nothing waits for)
    wg_cols(n, false, W, n, [&](int i, int j, double v) { gA[j + (int64_t)i * n] = v; });
    gsync();
    wg_trsm_ln(n, bw, n, L, n, A, n, s);  // A = L^-1 K L^-T
    // exactly symmetric: the upper triangle from the lower one
    wg_cols(n, true, A, n, [&](int i, int j, double v) { gA[j + (int64_t)i * n] = v; });
    gsync();
    if (n >= SYTRD_BLK_MIN)
        wg_sytrd_blk(n, A, n, p.tau, p.U, s);
    else
        wg_sytrd(n, A, n, p.tau, s);
    const int dc = wg_stedc(n, Z, n, W, p.U, p.Y, p.R, s);
    gsync();
    if (dc) return -(int64_t)dc;
    wg_ormtr(n, A, n, p.tau, Z, n, W, s);
    wg_trsm_lt(n, bw, n, L, n, Z, n, s);  // V = L^-T Z
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
    gdouble* gV = (gdouble*)p.V;
    wg_cols(n, false, Z, n, [&](int i, int j, double v) { gV[i + (int64_t)s.rk[j] * ld] = v; });
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

// A launch in flight: its workspace and the problems it writes.
struct fl_batch {
    fl_ctx* ctx = nullptr;
    hipStream_t s = nullptr;
    std::vector<fl_op*> ops;
    DevBuf bws, bprobs, border, bnext, bstat;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~fl_batch() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

extern "C" int fl_eigensolve_batched_begin(fl_ctx* ctx, int64_t count, fl_op* const* ops, int precision,
                                           fl_batch** out) {
    if (!ctx) return FL_EINVAL;
    if (!out) return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_batched: bad arguments");
    *out = nullptr;
    if (count < 0 || (count > 0 && !ops)) return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_batched: bad arguments");
    if (precision != FL_FP64)
        return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_batched: the batched solver runs in FP64 only");
    if (count == 0) return FL_OK;
    if (count > (int64_t)1 << 30) return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_batched: too many problems");
    for (int64_t i = 0; i < count; ++i) {
        const fl_op* op = ops[i];
        if (!op || op->device != ctx->device)
            return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_batched: null operator or operator of another device");
        if (!op->K || !op->M)
            return fl_fail(ctx, FL_ESTATE, "fl_eigensolve_batched: an operator holds no dense pencil");
        if (op->n < 1 || op->n > NMAX)
            return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_batched: each n must be in [1, 1024]");
        for (int64_t j = 0; j < i; ++j)
            if (ops[j] == op) return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_batched: an operator appears twice");
    }
    FL_HIP(ctx, hipSetDevice(ctx->device));
    auto bt = std::make_unique<fl_batch>();
    fl_batch& B = *bt;
    B.ctx = ctx;
    B.s = ctx->stream;
    B.ops.assign(ops, ops + count);
    hipStream_t s = B.s;
    // workspace: L, W, A, Z and tau per problem, 256-byte aligned
    std::vector<int64_t> off(count);
    int64_t tot = 0;
    auto al = [](int64_t x) { return (x + 31) / 32 * 32; };
    for (int64_t i = 0; i < count; ++i) {
        const int64_t n = ops[i]->n;
        const int64_t wsz = ormtr_wsz(n);
        off[i] = tot;
        tot += al(n * n) * 5 + al(wsz) + al(4 * n) + al(n);
    }
    FL_HIP(ctx, B.bws.alloc(sizeof(double) * tot));
    std::vector<BProb> hp(count);
    for (int64_t i = 0; i < count; ++i) {
        fl_op* op = ops[i];
        const int64_t n = op->n;
        if (!op->theta) FL_HIP(ctx, hipMalloc(&op->theta, sizeof(double) * n));
        if (!op->logtheta) FL_HIP(ctx, hipMalloc(&op->logtheta, sizeof(double) * n));
        if (!op->V) FL_HIP(ctx, hipMalloc(&op->V, sizeof(double) * op->ld * n));
        op->has_eig = 0;
        double* w = B.bws.as<double>() + off[i];
        const int64_t wsz = ormtr_wsz(n);
        BProb& b = hp[i];
        b.n = n;
        b.ld = op->ld;
        {
            int64_t bw = -1;
            int rcb = fl_pattern_bandwidth(op, &bw);
            if (rcb) return rcb;
            b.bw = bw >= 0 ? bw : n - 1;  // no pattern: dense
        }
        b.K = op->K;
        b.M = op->M;
        b.V = op->V;
        b.theta = op->theta;
        b.logtheta = op->logtheta;
        b.L = w;
        b.A = w + al(n * n);
        b.Z = w + 2 * al(n * n);
        b.W = w + 3 * al(n * n);
        b.U = b.W + al(wsz);
        b.Y = b.U + al(n * n);
        b.R = b.Y + al(n * n);
        b.tau = b.R + al(4 * n);
    }
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ops[a]->n > ops[b]->n; });
    FL_HIP(ctx, B.bprobs.alloc(sizeof(BProb) * count));
    FL_HIP(ctx, B.border.alloc(sizeof(int) * count));
    FL_HIP(ctx, B.bnext.alloc(sizeof(unsigned)));
    FL_HIP(ctx, B.bstat.alloc(sizeof(int64_t) * count));
    // (pageable sources: the copies complete before these calls return)
    FL_HIP(ctx, hipMemcpyAsync(B.bprobs.p, hp.data(), sizeof(BProb) * count, hipMemcpyHostToDevice, s));
    FL_HIP(ctx, hipMemcpyAsync(B.border.p, order.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
    FL_HIP(ctx, hipMemsetAsync(B.bnext.p, 0, sizeof(unsigned), s));
    FL_HIP(ctx, hipMemsetAsync(B.bstat.p, 0, sizeof(int64_t) * count, s));
    int cus = 256;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) cus = prop.multiProcessorCount;
    }
    const unsigned grid = (unsigned)std::min<int64_t>(count, 2 * (int64_t)cus);
    FL_HIP(ctx, hipEventCreate(&B.e0));
    FL_HIP(ctx, hipEventCreate(&B.e1));
    FL_HIP(ctx, hipEventRecord(B.e0, s));
    {
        KScope ks("batched_eig", s);
        batched_eig_kernel<<<grid, BT, 0, s>>>(B.bprobs.as<BProb>(), B.border.as<int>(), (int)count,
                                               B.bnext.as<unsigned>(), B.bstat.as<int64_t>());
    }
    FL_HIP(ctx, hipGetLastError());
    FL_HIP(ctx, hipEventRecord(B.e1, s));
    *out = bt.release();
    return FL_OK;
}

extern "C" int fl_eigensolve_batched_wait(fl_batch* b, fl_eig_info* infos) {
    if (!b) return FL_OK;
    std::unique_ptr<fl_batch> own(b);
    fl_ctx* ctx = b->ctx;
    FL_HIP(ctx, hipSetDevice(ctx->device));
    const int64_t count = (int64_t)b->ops.size();
    FL_HIP(ctx, hipEventSynchronize(b->e1));
    std::vector<int64_t> st(count);
    FL_HIP(ctx, hipMemcpyAsync(st.data(), b->bstat.p, sizeof(int64_t) * count, hipMemcpyDeviceToHost, b->s));
    FL_HIP(ctx, hipStreamSynchronize(b->s));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, b->e0, b->e1);
    int rc = FL_OK;
    for (int64_t i = 0; i < count; ++i) {
        fl_op* op = b->ops[i];
        int code = FL_OK;
        if (st[i] > 0) code = FL_ENOTSPD;
        if (st[i] < 0) code = FL_ENOCONV;
        if (code == FL_OK) {
            op->has_eig = 1;
            op->eig_precision = FL_FP64;
            op->refine_iters = 0;
            op->refine_resid = 0.0;
        }
        if (infos) {
            infos[i] = fl_eig_info{};
            infos[i].status = code;
            infos[i].index = st[i] > 0 ? st[i] : (st[i] < 0 ? -st[i] : 0);
            infos[i].total_ms = ms;
            const double n = (double)op->n;
            infos[i].flops_nominal = 9.0 * n * n * n;
        }
        if (code != FL_OK && rc == FL_OK) {
            rc = code;
            fl_fail(ctx, code,
                    std::string("fl_eigensolve_batched: problem ") + std::to_string(i) +
                        (code == FL_ENOTSPD ? ": M is not positive definite at pivot "
                                            : ": the tridiagonal eigensolver did not converge, code ") +
                        std::to_string(st[i] > 0 ? st[i] : -st[i]));
        }
    }
    return rc;
}

extern "C" int fl_eigensolve_batched(fl_ctx* ctx, int64_t count, fl_op* const* ops, int precision,
                                     fl_eig_info* infos) {
    if (!ctx) return FL_EINVAL;
    fl_batch* b = nullptr;
    const int rc = fl_eigensolve_batched_begin(ctx, count, ops, precision, &b);
    if (rc != FL_OK) return rc;
    return fl_eigensolve_batched_wait(b, infos);
}
