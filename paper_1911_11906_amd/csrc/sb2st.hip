// Stage 2 of the two-stage tridiagonalisation: symmetric band (width b) ->
// tridiagonal by bulge chasing.
//
// Sweep i annihilates column i below its subdiagonal with a Householder
// reflector on rows R_0 = [i+1, i+b]; applying it from the right to the
// block below creates a bulge, whose first column is annihilated by the next
// reflector on rows R_1 = [i+b+1, i+2b], and so on down the band.  Only the
// first column of each bulge is removed; the rest is removed by later sweeps,
// so the working band holds 2b sub-diagonals.  Task (i, j) touches
// the blocks (R_j, R_{j-1}), (R_j, R_j) and (R_{j+1}, R_j); the blocks of task
// (i-1, j') are the same blocks shifted up by one row and column, which meet
// those of (i, j) only for j' in [j-1, j+2].  With (i-1, j+2) they share a
// single element: the first entry of the column that (i-1, j+2) annihilates
// (which becomes its beta), the last row and column of (i, j)'s block below.
// So (i, j) may start once sweep i-1 has finished task j+1 and task j+2 has
// formed its reflector and stored that column: each task publishes the
// annihilated column right after its Householder step (progx) and the rest
// of its blocks at its end (prog); the final write-back skips that column.
//
// One persistent cooperative launch: workgroup w runs sweeps w, w+G, ...;
// each task stages its three b x b blocks in LDS; per-sweep progress
// counters are published with agent-scope release and read with acquire
// (they order the band traffic across the XCD L2 caches).
#include "internal.h"

namespace {

constexpr int BMAX = 64;  // (index arithmetic below uses BMAX = 64 = 1 << 6)
constexpr int LDB = BMAX + 1;
constexpr int NTH = 1024;

__device__ inline int64_t ntasks(int64_t n, int b, int64_t i) { return 1 + (n - 3 - i) / b; }

__device__ inline double band_get(const double* AB, int64_t ldab, int64_t r, int64_t c) {
    return AB[(r - c) + c * ldab];
}

constexpr long SPIN_CAP = 20000000;  // bounded wait: every wave exits even if a predecessor stalls

__global__ __launch_bounds__(NTH) void sb2st_kernel(int64_t n, int b, double* AB, int64_t ldab, double* V2,
                                                    double* tau2, int64_t maxt, int* prog, int* progx, int* abort) {
    __shared__ double bufA[BMAX * LDB], bufB[BMAX * LDB];  // off-diagonal / below blocks (rotate roles)
    __shared__ double S[BMAX * LDB];                        // symmetric diagonal block (full)
    __shared__ double vv[BMAX], pv[BMAX], wv[BMAX], pb[BMAX];
    constexpr int NG = NTH / 64;  // row groups of the products
    __shared__ double red[NG][BMAX], redS[NG][BMAX], redB[NG][BMAX];
    __shared__ double sc[4];
    __shared__ int quit;
    const int t = threadIdx.x;
    const int64_t nsweeps = n - 2;
    for (int64_t i = blockIdx.x; i < nsweeps; i += gridDim.x) {
        const int64_t nt = ntasks(n, b, i);
        const int64_t ntp = (i > 0) ? ntasks(n, b, i - 1) : 0;
        double* Boff = bufA;
        double* Bbl = bufB;
        for (int64_t j = 0; j < nt; ++j) {
            // ---- wait for sweep i-1 to clear our region (bounded)
            if (t == 0) {
                quit = 0;
                if (i > 0) {
                    const int need = (int)((j + 2 < ntp) ? (j + 2) : ntp);
                    const int needx = (int)((j + 3 < ntp) ? (j + 3) : ntp);
                    long spins = 0;
                    // poll relaxed (no cache invalidation per poll), acquire once
                    while (__hip_atomic_load(&prog[i - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need ||
                           __hip_atomic_load(&progx[i - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < needx) {
                        __builtin_amdgcn_s_sleep(2);
                        if (++spins > SPIN_CAP || __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            quit = 1;
                            break;
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
            }
            __syncthreads();
            if (quit) return;
            const int64_t r0 = i + 1 + j * b;
            const int L = (int)((n - r0) < b ? (n - r0) : b);          // rows of R_j
            const int64_t q0 = r0 + L;
            const int Lb = (int)(q0 < n ? ((n - q0) < b ? (n - q0) : b) : 0);  // rows of R_{j+1}
            const int64_t c0 = r0 - b;                                   // first column of R_{j-1}
            // ---- load: x (j == 0: column i), S = A[R_j, R_j], Bbl = A[R_{j+1}, R_j].
            // All global loads of the task are issued into registers before any
            // LDS store, so their latencies overlap instead of adding up.
            {
                constexpr int PER = (BMAX * BMAX + NTH - 1) / NTH;  // elements per thread per block
                double sv[PER], bv[PER];
                double xv = 0.0;
                if (j == 0 && t < L) xv = band_get(AB, ldab, r0 + t, i);
#pragma unroll
                for (int q = 0; q < PER; ++q) {
                    const int e = t + q * NTH;
                    const int r = e % BMAX, c = e / BMAX;
                    sv[q] = (r < L && c < L && r >= c) ? band_get(AB, ldab, r0 + r, r0 + c) : 0.0;
                    bv[q] = (r < Lb && c < L) ? band_get(AB, ldab, q0 + r, r0 + c) : 0.0;
                }
                if (j == 0 && t < L) Boff[t] = xv;
#pragma unroll
                for (int q = 0; q < PER; ++q) {
                    const int e = t + q * NTH;
                    const int r = e % BMAX, c = e / BMAX;
                    if (r < L && c < L && r >= c) {
                        S[r + c * LDB] = sv[q];
                        S[c + r * LDB] = sv[q];
                    }
                    if (r < Lb && c < L) Bbl[r + c * LDB] = bv[q];
                }
            }
            __syncthreads();
            // ---- Householder of x = Boff[:, 0] (length L), by wave 0, which
            // also writes v and replaces x by (beta, 0, ..., 0)
            if (t < 64) {
                const double xr = (t < L) ? Boff[t] : 0.0;
                double s2 = (t >= 1) ? xr * xr : 0.0;
                for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off, 64);
                const double x0 = __shfl(xr, 0, 64);
                double beta, tauc, scale;
                if (s2 == 0.0 || L < 2) {
                    beta = x0;
                    tauc = 0.0;
                    scale = 0.0;
                } else {
                    const double nrm = sqrt(x0 * x0 + s2);
                    beta = (x0 >= 0.0) ? -nrm : nrm;
                    tauc = (beta - x0) / beta;
                    scale = 1.0 / (x0 - beta);
                }
                vv[t] = (t == 0) ? 1.0 : (t < L ? xr * scale : 0.0);
                const double xn = (t == 0) ? beta : 0.0;
                if (t < L) Boff[t] = xn;
                if (t == 0) sc[1] = tauc;
                // publish the annihilated column (column i for j = 0, else the
                // first column of the block left of R_j): wave 0 waits for its
                // own stores, then releases them with the flag
                if (t < L) {
                    const int64_t col = (j == 0) ? i : c0;
                    AB[(r0 + t - col) + col * ldab] = xn;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_s_waitcnt(0);
                if (t == 0) __hip_atomic_store(&progx[i], (int)(j + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();
            const double tauc = sc[1];
            if (tauc != 0.0) {
                // ---- the three products with v, one phase (4 row groups x 64 lanes):
                // left  wv_c = v^T Boff[:, c] (c >= 1, j >= 1)
                // sym   pv = S v
                // right pb = Bbl v
                const int lane = t & 63, grp = t >> 6;
                {
                    double sl = 0.0, ss = 0.0, sb = 0.0;
                    if (j > 0 && lane >= 1 && lane < b)
                        for (int r = grp; r < L; r += NG) sl += vv[r] * Boff[r + lane * LDB];
                    if (lane < L)
                        for (int c = grp; c < L; c += NG) ss += S[lane + c * LDB] * vv[c];
                    if (lane < Lb)
                        for (int c = grp; c < L; c += NG) sb += Bbl[lane + c * LDB] * vv[c];
                    red[grp][lane] = sl;
                    redS[grp][lane] = ss;
                    redB[grp][lane] = sb;
                }
                __syncthreads();
                // ---- combine (wave 0): wv, w = p - (tau/2)(v^T p) v with p = tau S v, pb
                if (t < 64) {
                    double sl = 0.0, ss = 0.0, sb = 0.0;
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        sl += red[g][t];
                        ss += redS[g][t];
                        sb += redB[g][t];
                    }
                    wv[t] = sl;
                    const double p = (t < L) ? tauc * ss : 0.0;
                    double a = vv[t] * p;
                    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
                    pv[t] = p - 0.5 * tauc * a * vv[t];
                    pb[t] = tauc * sb;
                }
                __syncthreads();
                // ---- the three updates
                // (r, c) = (e mod 64, e / 64): power-of-two indexing, no runtime divisions
                for (int e = t; e < BMAX * BMAX; e += NTH) {
                    const int r = e & (BMAX - 1), c = e >> 6;
                    if (j > 0 && r < L && c >= 1 && c < b) Boff[r + c * LDB] -= tauc * vv[r] * wv[c];
                    if (r < L && c < L) S[r + c * LDB] -= vv[r] * pv[c] + pv[r] * vv[c];
                    if (r < Lb && c < L) Bbl[r + c * LDB] -= pb[r] * vv[c];
                }
            }
            __syncthreads();
            // ---- write back (the annihilated column went out with progx)
            for (int e = t; e < BMAX * BMAX; e += NTH) {
                const int r = e & (BMAX - 1), c = e >> 6;
                if (j > 0 && r < L && c >= 1 && c < b) AB[(r0 + r - (c0 + c)) + (c0 + c) * ldab] = Boff[r + c * LDB];
                if (r < L && c < L && r >= c) AB[(r - c) + (r0 + c) * ldab] = S[r + c * LDB];
                if (r < Lb && c < L) AB[(q0 + r - (r0 + c)) + (r0 + c) * ldab] = Bbl[r + c * LDB];
            }
            double* vout = V2 + (i * maxt + j) * (int64_t)b;
            // reflectors are read only by the back-transform, after the
            // launch: written through to memory (system-scope relaxed
            // stores) so that the per-task release has no dirty lines of
            // them to write back
            for (int r = t; r < b; r += NTH)
                __hip_atomic_store(&vout[r], (r < L) ? vv[r] : 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            if (t == 0) __hip_atomic_store(&tau2[i * maxt + j], tauc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            // ---- publish progress: every wave first waits for its own stores
            // (a plain workgroup barrier waits for LDS traffic only), then
            // thread 0's agent-scope release writes the L2 back and sets the flag
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_s_barrier();
            if (t == 0) __hip_atomic_store(&prog[i], (int)(j + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            // the block below becomes the next off-diagonal block
            double* tmp = Boff;
            Boff = Bbl;
            Bbl = tmp;
        }
    }
}

// ---------------------------------------------------------------------------
// Stationary bulge chase for b = 64.  Workgroup j owns the rows
// R_j(i) = [i+1+jb, i+(j+1)b] of every sweep i: the symmetric block
// S_j = A[R_j, R_j] and the block to its left B_j = A[R_j, R_{j-1}] stay in
// LDS for the whole launch.  Task (i, j) is then
//   B_j := B_j H_{i,j-1}                     (right reflector of task (i, j-1))
//   H_{i,j} from column 0 of B_j             (column i itself for j = 0)
//   B_j := H_{i,j} B_j,  S_j := H_{i,j} S_j H_{i,j}
// and the only data crossing workgroups are the reflector (to j+1) and, for
// the move of every block down by one row and column at the next sweep, the
// first row of B_j and S_j (to j-1): the dropped row/column of S_j becomes
// the new last column of B_j, the new last row/column of S_j is workgroup
// j+1's first row, and the new last row of B_j is zero except for j+1's
// beta.  A ring index (logical row r at physical (r + i) mod 64) makes that
// move free.  Every task (i, j) reads only tasks (i, j-1) and (i-1, j+1),
// so all of them are ready by t = 2i + j and the launch is a wavefront of
// 2n steps, each one message hand-off long.
//
// Hand-off without flags: every message word is written once (reflectors go
// straight to their place in V2 / tau2, rows to RM), all of them pre-filled
// with a signalling-NaN sentinel that arithmetic never produces; the reader
// polls the words themselves with agent-scope relaxed atomics, which bypass
// the non-coherent caches, so no release/acquire fence (and no L2 write-back
// or invalidation) is on the chain.
constexpr int RB = 64;
constexpr int RLD = RB + 1;
constexpr int RTH = 256;
constexpr long long RING_SENTINEL = 0x7FF4A5A5A5A5A5A5ll;
constexpr long RING_SPIN_CAP = 4000000;

__device__ inline bool ring_unset(double v) { return __double_as_longlong(v) == RING_SENTINEL; }

// One wave polls the 64 words at p (lane k: p[k]) and the word px until none
// holds the sentinel; false if the wait was abandoned (abort raised).
__device__ bool ring_poll(const double* p, const double* px, int lane, double& a, double& x, int* abort) {
    for (long spins = 0;; ++spins) {
        a = __hip_atomic_load(p + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = __hip_atomic_load(px, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__all(!ring_unset(a) && !ring_unset(x))) return true;
        if ((spins & 63) == 63) {
            const int ab = __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__any(ab != 0) || spins > RING_SPIN_CAP) {
                if (lane == 0) __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

__device__ inline void ring_put(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(RTH) void chase_ring_kernel(int64_t n, const double* __restrict__ AB, int64_t ldab,
                                                         double* d, double* e, double* V2, double* tau2, int64_t maxt,
                                                         double* RM, int64_t nwg, int* abort) {
    __shared__ double S[RB * RLD], Bk[RB * RLD];
    __shared__ double vin[RB], vv[RB], wvec[RB], msg[RB + 1];
    __shared__ double red[RTH / 64][RB], red2[RTH / 64][RB];
    __shared__ double tin_s, tau_s;
    __shared__ int quit;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t j = blockIdx.x;
    // sweep 0: S_j = A[R_j, R_j], B_j = A[R_j, R_{j-1}] (band rows only; zero
    // beyond the matrix), ring offset 0
    {
        const int64_t r00 = 1 + j * RB;
        for (int q = t; q < RB * RB; q += RTH) {
            const int r = q & (RB - 1), c = q >> 6;
            const int64_t gr = r00 + r, gc = r00 + c, gb = r00 - RB + c;
            double sv = 0.0, bv = 0.0;
            if (gr < n && gc < n) sv = (gr >= gc) ? AB[(gr - gc) + gc * ldab] : AB[(gc - gr) + gr * ldab];
            if (gr < n && gb >= 0 && r <= c) bv = AB[(gr - gb) + gb * ldab];
            S[r + c * RLD] = sv;
            Bk[r + c * RLD] = bv;
        }
        if (j == 0 && t == 0) d[0] = AB[0];
        if (t == 0) quit = 0;
    }
    __syncthreads();
    const int64_t last = n - 2 - j * RB;  // the last sweep whose R_j starts inside the matrix
    for (int64_t i = 0; i <= last; ++i) {
        const int off = (int)(i & (RB - 1));      // physical index of logical row / column 0
        const int q = (off + RB - 1) & (RB - 1);  // physical index of logical row / column b - 1
        const int64_t r0 = i + 1 + j * RB;
        const int L = (int)((n - r0) < RB ? (n - r0) : RB);
        // ---- inputs: wave 0 the reflector of task (i, j-1), wave 1 the first
        // row of task (i-1, j+1) (zero when R_{j+1} lay beyond the matrix)
        if (wave == 0 && j > 0) {
            double a, x;
            if (!ring_poll(V2 + (i * maxt + (j - 1)) * RB, tau2 + i * maxt + (j - 1), lane, a, x, abort)) {
                if (lane == 0) quit = 1;
            } else {
                vin[(lane + off) & (RB - 1)] = a;
                if (lane == 0) tin_s = x;
            }
        }
        if (wave == 1 && i > 0) {
            if (i + (j + 1) * RB <= n - 1) {
                const double* pm = RM + ((i - 1) * nwg + (j + 1)) * (RB + 1);
                double a, x;
                if (!ring_poll(pm, pm + RB, lane, a, x, abort)) {
                    if (lane == 0) quit = 1;
                } else {
                    msg[lane] = a;
                    if (lane == 0) msg[RB] = x;
                }
            } else {
                msg[lane] = 0.0;
                if (lane == 0) msg[RB] = 0.0;
            }
        }
        __syncthreads();
        if (quit) return;
        // ---- move down one row and column: physical q leaves as logical 0
        // and comes back as logical b - 1
        if (i > 0) {
            if (t < RB) {
                if (t != q) {
                    const double old = S[t + q * RLD];
                    const double nv = msg[(t - q) & (RB - 1)];
                    Bk[t + q * RLD] = old;
                    Bk[q + t * RLD] = 0.0;
                    S[t + q * RLD] = nv;
                    S[q + t * RLD] = nv;
                } else {
                    if (j == 0) d[i] = S[q + q * RLD];
                    Bk[q + q * RLD] = msg[0];
                    S[q + q * RLD] = msg[RB];
                }
            }
            __syncthreads();
        }
        // ---- right reflector of task (i, j-1): B := B - tau (B v) v^T
        if (j > 0) {
            const double ti = tin_s;
            double part = 0.0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int c = wave * 16 + k;
                part += Bk[lane + c * RLD] * vin[c];
            }
            red[wave][lane] = part;
            __syncthreads();
            if (ti != 0.0) {
                const double w = ti * (red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane]);
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const int c = wave * 16 + k;
                    Bk[lane + c * RLD] -= w * vin[c];
                }
            }
            __syncthreads();
        }
        // ---- Householder of the target column (logical 0; for j = 0 the
        // column i itself, logical b - 1), by wave 0; the reflector goes out
        // at once
        const int tc = (j == 0) ? q : off;
        if (wave == 0) {
            const int lr = (lane - off) & (RB - 1);
            const double xr = (lr < L) ? Bk[lane + tc * RLD] : 0.0;
            double s2 = (lr >= 1) ? xr * xr : 0.0;
            for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, 64);
            const double x0 = __shfl(xr, off, 64);
            double beta, tau, scale;
            if (s2 == 0.0 || L < 2) {
                beta = x0;
                tau = 0.0;
                scale = 0.0;
            } else {
                const double nrm = sqrt(x0 * x0 + s2);
                beta = (x0 >= 0.0) ? -nrm : nrm;
                tau = (beta - x0) / beta;
                scale = 1.0 / (x0 - beta);
            }
            const double v = (lr == 0) ? 1.0 : (lr < L ? xr * scale : 0.0);
            vv[lane] = v;
            Bk[lane + tc * RLD] = (lr == 0) ? beta : 0.0;
            if (L >= 2) {
                ring_put(V2 + (i * maxt + j) * RB + lr, v);
                if (lane == 0) ring_put(tau2 + i * maxt + j, tau);
            }
            if (lane == 0) {
                tau_s = tau;
                if (j == 0) e[i] = beta;
            }
        }
        __syncthreads();
        // ---- left reflector on B (columns other than the target) and the
        // two-sided update of S, column c = lane, rows 16 wave .. 16 wave + 15
        const double tau = tau_s;
        if (tau != 0.0) {
            double pl = 0.0, ps = 0.0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int r = wave * 16 + k;
                const double vr = vv[r];
                if (j > 0) pl += vr * Bk[r + lane * RLD];
                ps += vr * S[r + lane * RLD];
            }
            red[wave][lane] = pl;
            red2[wave][lane] = ps;
            __syncthreads();
            // y_c = v^T B[:, c];  p = tau S v;  w = p - (tau / 2)(v^T p) v
            const double y = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
            const double p = tau * (red2[0][lane] + red2[1][lane] + red2[2][lane] + red2[3][lane]);
            double a = vv[lane] * p;
            for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
            const double w = p - 0.5 * tau * a * vv[lane];
            if (wave == 0) wvec[lane] = w;
            __syncthreads();
            const double vc = vv[lane];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int r = wave * 16 + k;
                const double vr = vv[r], wr = wvec[r];
                if (j > 0 && lane != tc) Bk[r + lane * RLD] -= tau * vr * y;
                S[r + lane * RLD] -= vr * w + wr * vc;
            }
        }
        // ---- first row out, for workgroup j-1's next sweep: (beta, B[0, 1..],
        // S[0, 0]); each word is read by the thread that last wrote it
        if (j > 0 && wave == (off >> 4)) {
            double* pm = RM + (i * nwg + j) * (RB + 1);
            ring_put(pm + ((lane - off) & (RB - 1)), Bk[off + lane * RLD]);
            if (lane == off) ring_put(pm + RB, S[off + off * RLD]);
        }
    }
    if (j == 0) {
        __syncthreads();
        if (t == 0) {
            const int o = (int)(last & (RB - 1));
            d[n - 1] = S[o + o * RLD];
        }
    }
}

__global__ void ring_fill_kernel(int64_t count, double* p) {
    const double s = __longlong_as_double(RING_SENTINEL);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = s;
}

__global__ void band_to_tridiag_kernel(int64_t n, const double* __restrict__ AB, int64_t ldab, double* d, double* e) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = AB[i * ldab];
    if (i < n - 1) e[i] = AB[1 + i * ldab];
}

}  // namespace

int64_t fl_sb2st_maxt(int64_t n, int b) { return n >= 3 ? 1 + (n - 3) / b : 1; }

int64_t fl_sb2st_ring_groups(int64_t n) { return n >= 3 ? 1 + (n - 2) / RB : 0; }
int64_t fl_sb2st_ring_msg_elems(int64_t n) { return n >= 3 ? (n - 1) * fl_sb2st_ring_groups(n) * (RB + 1) : 0; }

// Whether the stationary chase can run: b = 64 and one workgroup per block
// column resident at once.
bool fl_sb2st_ring_fits(int64_t n, int b) {
    if (b != RB || n < 3) return false;
    int dev = 0, per = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, chase_ring_kernel, RTH, 0) != hipSuccess) return false;
    return fl_sb2st_ring_groups(n) <= (int64_t)per * p.multiProcessorCount;
}

// The stationary chase (b = 64): d, e and the reflectors V2 / tau2 (the same
// layout as fl_sb2st); RM: fl_sb2st_ring_msg_elems(n) doubles of row
// messages.  AB is only read.  V2, tau2 and RM are filled with the sentinel
// first (on s), so no word of an earlier call can be taken for a message.
hipError_t fl_sb2st_ring(hipStream_t s, int64_t n, const double* AB, int64_t ldab, double* d, double* e, double* V2,
                         double* tau2, double* RM, int* abort) {
    const int64_t maxt = fl_sb2st_maxt(n, RB), nsw = n - 2, nwg = fl_sb2st_ring_groups(n);
    ring_fill_kernel<<<2048, 256, 0, s>>>(nsw * maxt * RB, V2);
    ring_fill_kernel<<<256, 256, 0, s>>>(nsw * maxt, tau2);
    ring_fill_kernel<<<2048, 256, 0, s>>>(fl_sb2st_ring_msg_elems(n), RM);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    int64_t nn = n, lda = ldab, mt = maxt, ng = nwg;
    void* args[] = {&nn, (void*)&AB, &lda, &d, &e, &V2, &tau2, &mt, &RM, &ng, &abort};
    KScope ks("sb2st", s);
    return hipLaunchCooperativeKernel((const void*)chase_ring_kernel, dim3((unsigned)nwg), dim3(RTH), args, 0, s);
}

// Band AB (lower, ld ldab >= 2b+1, zero below the first b+1 diagonals) ->
// d, e.  V2 (n-2 sweeps x maxt tasks x b) and tau2 receive the reflectors.
// prog: 2n ints of scratch; abort: device flag raised if a wait was abandoned.
hipError_t fl_sb2st(hipStream_t s, int64_t n, int b, double* AB, int64_t ldab, double* d, double* e, double* V2,
                    double* tau2, int* prog, int grid, int* abort) {
    hipError_t err;
    if (n >= 3 && b > 1) {
        if ((err = hipMemsetAsync(prog, 0, sizeof(int) * 2 * n, s)) != hipSuccess) return err;
        int64_t maxt = fl_sb2st_maxt(n, b);
        int64_t nsw = n - 2;
        unsigned G = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nsw, grid));
        int64_t nn = n, lda = ldab, mt = maxt;
        int bb = b;
        int* progx = prog + n;
        void* args[] = {&nn, &bb, &AB, &lda, &V2, &tau2, &mt, &prog, &progx, &abort};
        {
            KScope ks("sb2st", s);
            err = hipLaunchCooperativeKernel((const void*)sb2st_kernel, dim3(G), dim3(NTH), args, 0, s);
        }
        if (err != hipSuccess) return err;
    }
    band_to_tridiag_kernel<<<(unsigned)FL_DIV_UP(n, 256), 256, 0, s>>>(n, AB, ldab, d, e);
    return hipGetLastError();
}
