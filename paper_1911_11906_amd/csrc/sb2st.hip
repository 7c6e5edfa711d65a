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

__global__ void band_to_tridiag_kernel(int64_t n, const double* __restrict__ AB, int64_t ldab, double* d, double* e) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = AB[i * ldab];
    if (i < n - 1) e[i] = AB[1 + i * ldab];
}

}  // namespace

int64_t fl_sb2st_maxt(int64_t n, int b) { return n >= 3 ? 1 + (n - 3) / b : 1; }

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
