// Stage 1 of the two-stage tridiagonalisation: symmetric full -> band.
//
// Panel p (columns c0 .. c0+b) is QR-factored below the band:
// A[c0+b:n, c0:c0+b] = (I - V T V^T) [R; 0].  The trailing block is then
// updated two-sidedly on the matrix cores:
//     X = A22 V T,  W = X - 1/2 V (T^T V^T X),  A22 -= V W^T + W V^T
// (the lower triangle by the matrix cores, the upper one copied from it).
// The rank-2b updates of up to QL consecutive panels are deferred and applied
// as one rank-2 QL b product (a k of 2 b = 128 leaves each output tile's
// load and store of C unamortised).  Until then the pending pairs (V_k, W_k)
// are kept side by side in [V W] and [W V] (absolute rows), and a panel sees
// the current matrix through them: its own columns get the pending update
// before the QR, and A22 V = A22_stale V - [V W] ([W V]^T V).
// The panel QR is one cooperative kernel: each workgroup keeps a 256-row slab
// of the panel in registers; per column (or pair of columns) one exchange
// shares the partial dot products (every workgroup then reduces them
// itself, in a fixed order, so the result is deterministic).  An exchange
// has a region of its own, written once and pre-filled with a
// signalling-NaN sentinel that arithmetic never produces: every workgroup
// polls the words themselves with agent-scope relaxed atomics (which bypass
// the non-coherent caches), so no counter, release or acquire (no L2
// write-back or invalidation) sits between two columns.
#include "internal.h"

namespace {

constexpr int PNT = 512;   // threads per panel workgroup (256-row slabs: every exchange is read by each
                           // workgroup in full, so fewer, larger slabs mean less exchange traffic)
constexpr int NGRP = PNT / 64;  // row groups (one wave each)
constexpr int PRPT = 32;   // panel rows per thread-row-group
constexpr int PROWS = NGRP * PRPT;  // rows per workgroup slab (NGRP groups of 64 column lanes)

constexpr long SPIN_CAP = 2000000;  // bounded wait: every wave exits even if a peer never arrives

// Exchange words: a signalling NaN of the element type marks "not yet written".
template <class T> struct Unset;
template <> struct Unset<double> {
    static constexpr long long bits = 0x7FF4A5A5A5A5A5A5ll;
    __device__ static double value() { return __longlong_as_double(bits); }
    __device__ static bool is(double v) { return __double_as_longlong(v) == bits; }
};
template <> struct Unset<float> {
    static constexpr int bits = 0x7FA5A5A5;
    __device__ static float value() { return __int_as_float(bits); }
    __device__ static bool is(float v) { return __float_as_int(v) == bits; }
};

template <class T>
__device__ inline void xput(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ inline T xget(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Words of exchange k: the partial sums of G workgroups (128 each), then
// rows c and c+1 of the panel (64 each).
__host__ __device__ inline int64_t exch_elems(int64_t G) { return G * 128 + 128; }

template <class T>
__global__ void unset_fill_kernel(int64_t count, T* p) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = Unset<T>::value();
}

// QR of the m x kb panel P (ld lda) with kref reflectors.  On exit P holds R
// on and above its diagonal and the reflectors below (LAPACK layout), Vx
// (ld ldv) the explicit unit-lower V (zeros above the diagonal), tau[c].
//
// Two reflectors per grid barrier where that is safe.  One exchange carries,
// besides s_j = x_c^T a_j (rows > c) and rows c, c+1, the Gram row
// g_j = a_{c+1}^T a_j (rows > c+1).  With reflector c = (tau, v, w) known,
// column c+1 after it and its products with the other updated columns follow
// exactly from these sums:
//     P_j = v^T a_j (rows > c+1) = scale (s_j - x_{c+1} a_j[c+1]),
//     Q   = v^T v   (rows > c+1) = scale^2 (|x|^2 - x_{c+1}^2),
//     s'_j = g_j - tau w_j P_{c+1} - tau w_{c+1} P_j + tau^2 w_{c+1} w_j Q,
// and |a'_{c+1}|^2 = s'_{c+1}.  That norm loses accuracy by the factor
// g_{c+1} / s'_{c+1}; every workgroup takes reflector c+1 from the exchange
// only if that factor is at most 1 / PAIR_MIN (and otherwise runs it in the
// next exchange as a single step), so its relative error stays below
// ~4 eps / PAIR_MIN.  The decision is made on the same reduced sums in every
// workgroup, in a fixed summation order: the result is deterministic.
//
// part: kref exchange regions of exch_elems(G) words, all unset on entry;
// abort: raised when a wait is abandoned (the result is then invalid).
constexpr double PAIR_MIN = 1.0 / 64;
template <class T>
__global__ __launch_bounds__(PNT) void panel_qr_kernel(int64_t m, int kb, int kref, T* P, int64_t lda, T* Vx,
                                                       int64_t ldv, T* tau, T* part, int* abort) {
    __shared__ T xc[PROWS];   // pivot column c (this slab's rows)
    __shared__ T xd[PROWS];   // column c+1: before reflector c (Gram row), after it (second update)
    __shared__ T red[NGRP][64], red2[NGRP][64];
    __shared__ T wv[64], gv[64];
    __shared__ T rows[128];  // rows c and c+1 of the panel
    __shared__ T sc[8];  // scale, tau, beta, | scale', tau', beta', pair flag
    const int t = threadIdx.x;
    const int lane = t & 63;   // panel column handled by this thread
    const int grp = t >> 6;    // row group
    const unsigned G = gridDim.x;
    const int64_t slab0 = (int64_t)blockIdx.x * PROWS;
    // rows of this thread: slab0 + grp + NGRP q, addressed from one base with
    // constant offsets (no per-row 64-bit addresses kept live)
    const int rows_here = (int)std::min<int64_t>(m - slab0, PROWS);
    const bool col_ok = lane < kb;
    T v[PRPT];
    {
        const T* Pb = P + (slab0 + grp) + (int64_t)(col_ok ? lane : 0) * lda;
#pragma unroll
        for (int q = 0; q < PRPT; ++q) v[q] = (grp + NGRP * q < rows_here && col_ok) ? Pb[NGRP * q] : T(0);
    }
    unsigned k = 0;  // exchanges so far
    for (int c = 0; c < kref;) {
        T* ex = part + (int64_t)k * exch_elems(G);
        const bool try2 = c + 1 < kref;
        // row indices relative to the slab: r = grp + NGRP q against the
        // slab-relative pivot lc (32-bit)
        const int lc = (int)std::max<int64_t>(-2, std::min<int64_t>(c - slab0, PROWS + 2));
        // pivot column (and column c+1) into LDS, zero at and above rows c
        // (c+1), so that every sum and update below runs over all rows
        if (lane == c) {
#pragma unroll
            for (int q = 0; q < PRPT; ++q) xc[grp + NGRP * q] = (grp + NGRP * q > lc) ? v[q] : T(0);
        }
        if (try2 && lane == c + 1) {
#pragma unroll
            for (int q = 0; q < PRPT; ++q) xd[grp + NGRP * q] = (grp + NGRP * q > lc + 1) ? v[q] : T(0);
        }
        __syncthreads();
        // partial sums over this slab: s_j (rows > c), g_j (rows > c+1); rows
        // beyond the panel hold zeros
        T s = T(0), g = T(0);
#pragma unroll
        for (int q = 0; q < PRPT; ++q) {
            s += xc[grp + NGRP * q] * v[q];
            g += xd[grp + NGRP * q] * v[q];
        }
        if (!try2) g = T(0);
        red[grp][lane] = s;
        red2[grp][lane] = g;
        // the workgroups owning rows c and c+1 publish them (v is indexed
        // with constants only, so that it stays in registers)
#pragma unroll
        for (int q = 0; q < PRPT; ++q) {
            const int64_t r = slab0 + grp + NGRP * q;
            if (r == c) xput(ex + G * 128 + lane, v[q]);
            if (try2 && r == c + 1) xput(ex + G * 128 + 64 + lane, v[q]);
        }
        __syncthreads();
        if (t < 64) {
            T* pw = ex + (size_t)blockIdx.x * 128;
            T a = T(0), a2 = T(0);
#pragma unroll
            for (int q = 0; q < NGRP; ++q) {
                a += red[q][t];
                a2 += red2[q][t];
            }
            xput(pw + t, a);
            xput(pw + 64 + t, a2);
        }
        __syncthreads();  // red is reused below
        ++k;
        // reduce the partials of all workgroups in a fixed order (the same in
        // every workgroup): row group q sums workgroups q, q+NGRP, ..., the
        // NGRP sums are added in LDS.  The words are polled RB workgroups at
        // a time (loads issued before any test), from clamped, always valid
        // addresses, until none is unset.
        int bad = 0;
        {
            constexpr int RB = 8;
            T acc = T(0), acc2 = T(0);
            const T* pp = ex + lane;
            for (unsigned w0 = (unsigned)grp; w0 < G && !bad; w0 += NGRP * RB) {
                T buf[RB], buf2[RB];
                for (long spins = 0;; ++spins) {
#pragma unroll
                    for (int q = 0; q < RB; ++q) {
                        const unsigned w = w0 + NGRP * q;
                        const size_t o = (size_t)(w < G ? w : 0) * 128;
                        buf[q] = xget(pp + o);
                        buf2[q] = xget(pp + o + 64);
                    }
                    bool ready = true;
#pragma unroll
                    for (int q = 0; q < RB; ++q)
                        ready = ready && (w0 + NGRP * q >= G || (!Unset<T>::is(buf[q]) && !Unset<T>::is(buf2[q])));
                    if (ready) break;
                    if ((spins & 63) == 63 &&
                        (spins > SPIN_CAP || __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                        __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        bad = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
#pragma unroll
                for (int q = 0; q < RB; ++q) {
                    acc += (w0 + NGRP * q < G) ? buf[q] : T(0);
                    acc2 += (w0 + NGRP * q < G) ? buf2[q] : T(0);
                }
            }
            red[grp][lane] = acc;
            red2[grp][lane] = acc2;
        }
        // rows c and c+1
        if (t < (try2 ? 128 : 64) && !bad) {
            T r;
            for (long spins = 0;; ++spins) {
                r = xget(ex + G * 128 + t);
                if (!Unset<T>::is(r)) break;
                if ((spins & 63) == 63 &&
                    (spins > SPIN_CAP || __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                    __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    bad = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            rows[t] = r;
        }
        if (__syncthreads_or(bad)) return;
        if (t < 64) {
            T a = T(0), a2 = T(0);
#pragma unroll
            for (int q = 0; q < NGRP; ++q) {
                a += red[q][t];
                a2 += red2[q][t];
            }
            wv[t] = a;
            gv[t] = a2;
        }
        __syncthreads();
        const T* r0v = rows;       // row c
        const T* r1v = rows + 64;  // row c+1
        if (t == 0) {
            const T x0 = r0v[c];
            const T sig = wv[c];  // |x(rows > c)|^2
            T beta, tauc, scale;
            if (sig == T(0)) {
                beta = x0;
                tauc = T(0);
                scale = T(0);
            } else {
                T nrm = sqrt(x0 * x0 + sig);
                beta = (x0 >= T(0)) ? -nrm : nrm;
                tauc = (beta - x0) / beta;
                scale = T(1) / (x0 - beta);
            }
            sc[0] = scale;
            sc[1] = tauc;
            sc[2] = beta;
            if (blockIdx.x == 0) tau[c] = tauc;
            int pair = 0;
            if (try2) {
                const T x1 = r1v[c];  // pivot column at row c+1
                const T v1 = scale * x1;
                const T w1 = r0v[c + 1] + scale * wv[c + 1];
                const T P1 = scale * (wv[c + 1] - x1 * r1v[c + 1]);
                const T Q = scale * scale * (sig - x1 * x1);
                const T gcc = gv[c + 1];
                const T sig2 = gcc - T(2) * tauc * w1 * P1 + tauc * tauc * w1 * w1 * Q;
                if (sig2 >= T(PAIR_MIN) * gcc) {
                    pair = 1;
                    const T y0 = r1v[c + 1] - tauc * v1 * w1;  // column c+1 at row c+1 after reflector c
                    T beta2, tau2, scale2;
                    if (!(sig2 > T(0))) {
                        beta2 = y0;
                        tau2 = T(0);
                        scale2 = T(0);
                    } else {
                        T nrm = sqrt(y0 * y0 + sig2);
                        beta2 = (y0 >= T(0)) ? -nrm : nrm;
                        tau2 = (beta2 - y0) / beta2;
                        scale2 = T(1) / (y0 - beta2);
                    }
                    sc[3] = scale2;
                    sc[4] = tau2;
                    sc[5] = beta2;
                    sc[6] = v1;
                    sc[7] = w1;
                    if (blockIdx.x == 0) tau[c + 1] = tau2;
                }
            }
            red[0][0] = (T)pair;
        }
        __syncthreads();
        const T scale = sc[0], tauc = sc[1], beta = sc[2];
        const bool pair = red[0][0] != T(0);
        // w_j = v^T a_j = a_j[c] + scale * s_j   (j > c)
        const T wj = (lane > c && lane < kb) ? (r0v[lane] + scale * wv[lane]) : T(0);
        // column c becomes (beta, reflector entries); columns j > c get
        // a_j -= tau v w_j with v = (1 at row c, scale x below)
        {
            const bool piv = lane == c;
            const T f = (lane > c && lane < kb) ? tauc * wj : T(0);
#pragma unroll
            for (int q = 0; q < PRPT; ++q) {
                const int r = grp + NGRP * q;
                const T vr = scale * xc[r] + (r == lc ? T(1) : T(0));
                const T pv = (r > lc) ? scale * v[q] : (r == lc ? beta : v[q]);
                v[q] = piv ? pv : v[q] - f * vr;
            }
        }
        if (!pair) {
            __syncthreads();
            c += 1;
            continue;
        }
        // reflector c+1 from the same exchange
        const T scale2 = sc[3], tau2 = sc[4], beta2 = sc[5], v1 = sc[6], w1 = sc[7];
        T wj2 = T(0);
        if (lane > c + 1 && lane < kb) {
            const T x1 = r1v[c];
            const T P1 = scale * (wv[c + 1] - x1 * r1v[c + 1]);
            const T Q = scale * scale * (wv[c] - x1 * x1);
            const T Pj = scale * (wv[lane] - x1 * r1v[lane]);
            const T s2 = gv[lane] - tauc * wj * P1 - tauc * w1 * Pj + tauc * tauc * w1 * wj * Q;
            wj2 = (r1v[lane] - tauc * v1 * wj) + scale2 * s2;
        }
        // column c+1 after reflector c, for the second update
        if (lane == c + 1) {
#pragma unroll
            for (int q = 0; q < PRPT; ++q) xd[grp + NGRP * q] = (grp + NGRP * q > lc + 1) ? v[q] : T(0);
        }
        __syncthreads();
        {
            const bool piv2 = lane == c + 1;
            const T f = (lane > c + 1 && lane < kb) ? tau2 * wj2 : T(0);
#pragma unroll
            for (int q = 0; q < PRPT; ++q) {
                const int r = grp + NGRP * q;
                const T vr = scale2 * xd[r] + (r == lc + 1 ? T(1) : T(0));
                const T pv = (r > lc + 1) ? scale2 * v[q] : (r == lc + 1 ? beta2 : v[q]);
                v[q] = piv2 ? pv : v[q] - f * vr;
            }
        }
        __syncthreads();
        c += 2;
    }
    // write back the factored panel and the explicit reflectors
    if (col_ok) {
        T* Pb = P + (slab0 + grp) + (int64_t)lane * lda;
        T* Vb = Vx + (slab0 + grp) + (int64_t)lane * ldv;
        const int ll = (int)std::max<int64_t>(-1, std::min<int64_t>(lane - slab0, PROWS));  // lane's diagonal row, slab-relative
#pragma unroll
        for (int q = 0; q < PRPT; ++q) {
            const int r = grp + NGRP * q;
            if (r < rows_here) {
                Pb[NGRP * q] = v[q];
                if (lane < kref) Vb[NGRP * q] = (r > ll) ? v[q] : (r == ll ? T(1) : T(0));
            }
        }
    }
}

// T (kref x kref upper, ld ldt) of the forward block reflector from the Gram
// matrix G = V^T V and tau: T_jj = tau_j, T(0:j, j) = -tau_j T(0:j,0:j) G(0:j, j).
// G is staged in LDS once; at step j, four lanes share row t < j, each summing
// every fourth term of its dot product, combined by two lane exchanges, so a
// step costs one barrier and at most 16 products per lane.
constexpr int LFT = 256;
template <class E>
__global__ __launch_bounds__(LFT) void larft_gram_kernel(int kref, const E* __restrict__ G, int64_t ldg,
                                                         const E* __restrict__ tau, E* T, int64_t ldt) {
    __shared__ E Ts[64 * 65];
    __shared__ E Gs[64 * 65];
    const int tid = threadIdx.x;
    for (int e = tid; e < 64 * 64; e += LFT) {
        const int r = e & 63, c = e >> 6;
        Gs[r + c * 65] = (r < kref && c < kref) ? G[r + c * ldg] : E(0);
        Ts[r + c * 65] = E(0);
    }
    __syncthreads();
    const int t = tid >> 2, part = tid & 3;  // row t, quarter part of its dot product
    for (int j = 0; j < kref; ++j) {
        E acc = E(0);
        if (t < j)
            for (int k = t + part; k < j; k += 4) acc += Ts[t + k * 65] * Gs[k + j * 65];
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        if (part == 0) {
            if (t < j) Ts[t + j * 65] = -tau[j] * acc;
            if (t == j) Ts[j + j * 65] = tau[j];
        }
        __syncthreads();
    }
    for (int e = tid; e < kref * kref; e += LFT) {
        const int r = e % kref, c = e / kref;
        T[r + c * ldt] = Ts[r + c * 65];
    }
}

// Band (lower, ld ldab, 2b+1 rows reserved) from the reduced matrix: the
// first b+1 diagonals, zeros below (room for the bulge-chasing fill).
template <class T>
__global__ void extract_band_kernel(int64_t n, int b, const T* __restrict__ A, int64_t lda, double* AB,
                                    int64_t ldab) {
    int64_t c = blockIdx.x;
    for (int d = threadIdx.x; d < ldab; d += blockDim.x) {
        double v = 0.0;
        if (d <= b && c + d < n) v = (double)A[(c + d) + c * lda];
        AB[d + c * ldab] = v;
    }
}

template <class T>
__global__ void copy_t_kernel(int64_t m, int64_t n, const T* __restrict__ A, int64_t lda, T* __restrict__ B,
                              int64_t ldb) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        if (i < m) B[i + j * ldb] = A[i + j * lda];
}

template <class T>
hipError_t copy_t(hipStream_t s, int64_t m, int64_t n, const T* A, int64_t lda, T* B, int64_t ldb) {
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 g((unsigned)FL_DIV_UP(m, 256), (unsigned)std::min<int64_t>(n, 65535));
    copy_t_kernel<T><<<g, 256, 0, s>>>(m, n, A, lda, B, ldb);
    return hipGetLastError();
}

}  // namespace
int64_t fl_sy2sb_panels(int64_t n, int b);
namespace {

constexpr int QL = 8;  // panels per deferred trailing update

template <class T>
hipError_t sy2sb_t(hipStream_t s, int64_t n, int b, T* A, int64_t lda, T* V1, int64_t ldv, T* T1, T* tau1, T* work,
                   T* part, int* abort) {
    const int64_t np = fl_sy2sb_panels(n, b);
    hipError_t e;
    const int64_t kw = 2 * (int64_t)QL * b;  // columns of [V W] and [W V]
    T* Gm = work;                            // b x b
    T* S = Gm + (int64_t)b * b;              // b x b
    T* R = S + (int64_t)b * b;               // b x b
    T* Y = R + (int64_t)b * b;               // n x b (ld m)
    T* X = Y + n * (int64_t)b;               // n x b (ld m)
    T* VW = X + n * (int64_t)b;              // n x kw (ld n), slot k: [V_k W_k]
    T* WV = VW + n * kw;                     // n x kw (ld n), slot k: [W_k V_k]
    T* Z = WV + n * kw;                      // kw x b (ld kw)
    int64_t p0 = 0;                          // first panel whose update is pending
    for (int64_t p = 0; p < np; ++p) {
        const int64_t c0 = p * b, r0 = c0 + b, m = n - r0;
        const int kb = b;
        const int kref = (int)std::min<int64_t>(b, m - 1);
        if (kref <= 0) break;
        const int64_t kp = 2 * (p - p0) * (int64_t)b;  // pending columns of [V W]
        // the panel's columns (diagonal block included) get the pending update
        if (kp > 0 && (e = fl_gemm_t(s, 0, 1, n - c0, kb, kp, -1.0, VW + c0, n, WV + c0, n, 1.0, A + c0 + c0 * lda,
                                     lda)))
            return e;
        T* Pn = A + r0 + c0 * lda;
        T* Vp = V1 + r0 + c0 * ldv;
        T* tp = tau1 + c0;
        const unsigned G = (unsigned)FL_DIV_UP(m, PROWS);
        {
            const int64_t fill = (int64_t)kref * exch_elems(G);
            unset_fill_kernel<T><<<(unsigned)std::min<int64_t>(FL_DIV_UP(fill, 256), 1024), 256, 0, s>>>(fill, part);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            int64_t mm = m;
            int kbb = kb, krf = kref;
            int64_t ldaa = lda, ldvv = ldv;
            void* args[] = {&mm, &kbb, &krf, &Pn, &ldaa, &Vp, &ldvv, &tp, &part, &abort};
            e = hipLaunchCooperativeKernel((const void*)panel_qr_kernel<T>, dim3(G), dim3(PNT), args, 0, s);
            if (e != hipSuccess) return e;
        }
        // T from G = V^T V
        T* Tp = T1 + p * (int64_t)b * b;
        e = fl_gemm_t(s, 1, 0, kref, kref, m, 1.0, Vp, ldv, Vp, ldv, 0.0, Gm, b);
        if (e != hipSuccess) return e;
        larft_gram_kernel<T><<<1, LFT, 0, s>>>(kref, Gm, b, tp, Tp, b);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // Y = A22 V with A22 = A[r0:n, r0:n] as of the last trailing update,
        // corrected by the pending pairs
        T* A22 = A + r0 + r0 * lda;
        if ((e = fl_gemm_t(s, 0, 0, m, kref, m, 1.0, A22, lda, Vp, ldv, 0.0, Y, m))) return e;
        if (kp > 0) {
            if ((e = fl_gemm_t(s, 1, 0, kp, kref, m, 1.0, WV + r0, n, Vp, ldv, 0.0, Z, kw))) return e;
            if ((e = fl_gemm_t(s, 0, 0, m, kref, kp, -1.0, VW + r0, n, Z, kw, 1.0, Y, m))) return e;
        }
        if ((e = fl_gemm_t(s, 0, 0, m, kref, kref, 1.0, Y, m, Tp, b, 0.0, X, m))) return e;      // X = Y T
        if ((e = fl_gemm_t(s, 1, 0, kref, kref, m, 1.0, Vp, ldv, X, m, 0.0, S, b))) return e;     // S = V^T X
        if ((e = fl_gemm_t(s, 1, 0, kref, kref, kref, 1.0, Tp, b, S, b, 0.0, R, b))) return e;   // R = T^T S
        // slot of this panel; a short last panel leaves columns of its slot
        // unwritten, which must then hold zeros
        T* vw = VW + kp * n;
        T* wv = WV + kp * n;
        if (kref < b) {
            for (T* q : {vw, wv}) {
                e = hipMemset2DAsync(q + r0, sizeof(T) * n, 0, sizeof(T) * m, 2 * b, s);
                if (e != hipSuccess) return e;
            }
        }
        // W = X - 1/2 V R, written straight into both slots
        if ((e = copy_t<T>(s, m, kref, X, m, vw + b * n + r0, n))) return e;
        if ((e = fl_gemm_t(s, 0, 0, m, kref, kref, -0.5, Vp, ldv, R, b, 1.0, vw + b * n + r0, n))) return e;
        if ((e = copy_t<T>(s, m, kref, Vp, ldv, vw + r0, n))) return e;
        if ((e = copy_t<T>(s, m, kref, vw + b * n + r0, n, wv + r0, n))) return e;
        if ((e = copy_t<T>(s, m, kref, Vp, ldv, wv + b * n + r0, n))) return e;
        // trailing update of the group: A[r0:n, r0:n] -= [V W] [W V]^T on the
        // tiles on and below the diagonal (the update is symmetric), then the
        // upper triangle from the lower one
        if (p + 1 - p0 == QL || p + 1 == np) {
            if ((e = fl_gemm_t(s, 0, 1, m, m, kp + 2 * b, -1.0, VW + r0, n, WV + r0, n, 1.0, A22, lda, 1))) return e;
            if ((e = fl_mirror_lower_t(s, m, A22, lda))) return e;
            p0 = p + 1;
        }
    }
    return hipSuccess;
}

}  // namespace

// Per-panel bookkeeping shared with the back-transform.
int64_t fl_sy2sb_panels(int64_t n, int b) {
    int64_t np = 0;
    for (int64_t c0 = 0; c0 + b < n - 1; c0 += b) ++np;
    return np;
}

// Reduce the symmetric A (full storage, ld lda) to band width b.  V1 (n x n,
// ld ldv) receives the explicit reflectors of every panel at the panel's own
// rows/columns (its entries above each panel must be zero on entry), T1 (np
// blocks of b x b) their T factors.  work: fl_sy2sb_work_elems(n, b) elements
// (about 4 QL n b); part: fl_sy2sb_part_elems(n) elements;
// abort: device flag raised if a cooperative wait was abandoned.
hipError_t fl_sy2sb(hipStream_t s, int64_t n, int b, double* A, int64_t lda, double* V1, int64_t ldv, double* T1,
                    double* tau1, double* work, double* part, int* abort) {
    return sy2sb_t<double>(s, n, b, A, lda, V1, ldv, T1, tau1, work, part, abort);
}
hipError_t fl_ssy2sb(hipStream_t s, int64_t n, int b, float* A, int64_t lda, float* V1, int64_t ldv, float* T1,
                     float* tau1, float* work, float* part, int* abort) {
    return sy2sb_t<float>(s, n, b, A, lda, V1, ldv, T1, tau1, work, part, abort);
}

int64_t fl_sy2sb_work_elems(int64_t n, int b) {
    const int64_t kw = 2 * (int64_t)QL * b;
    return 3 * (int64_t)b * b + 2 * n * (int64_t)b + 2 * n * kw + kw * b;
}
// exchange regions of the panel QR: at most 64 exchanges of a panel of at
// most ceil(n / PROWS) workgroups
int64_t fl_sy2sb_part_elems(int64_t n) { return 64 * exch_elems(FL_DIV_UP(n, PROWS)); }

hipError_t fl_extract_band(hipStream_t s, int64_t n, int b, const double* A, int64_t lda, double* AB, int64_t ldab) {
    if (n <= 0) return hipSuccess;
    extract_band_kernel<double><<<(unsigned)n, 128, 0, s>>>(n, b, A, lda, AB, ldab);
    return hipGetLastError();
}
hipError_t fl_extract_band_f(hipStream_t s, int64_t n, int b, const float* A, int64_t lda, double* AB, int64_t ldab) {
    if (n <= 0) return hipSuccess;
    extract_band_kernel<float><<<(unsigned)n, 128, 0, s>>>(n, b, A, lda, AB, ldab);
    return hipGetLastError();
}
