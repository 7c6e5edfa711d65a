// Back-transformation of the tridiagonal eigenvectors: Z := Q1 Q2 Z.
//
// Q2 (bulge chasing) is the product, in generation order, of the reflectors
// H(i, j) of sweep i, task j, acting on rows [i+1+jb, i+(j+1)b].  Reflectors
// of different sweeps overlap only as (i, j) with (i+d, j) (d < b) or
// (i+d, j-1) (1 <= d < 2b), so for a group of b consecutive sweeps the
// product equals prod_j-descending B(G, j) with B(G, j) = H(g, j) ... H(g+b-1, j),
// a (2b-1) x b staircase block reflector I - V T V^T.  Applying Q2: groups
// last to first, within a group j ascending.  Each workgroup owns a 32-column
// slab of Z and runs W = V^T Z, W = T W, Z -= V W on the matrix cores from LDS.
//
// Q1 (band reduction) is applied panel by panel, last first, with GEMMs.
#include "internal.h"
#include "gemm_tile.h"

namespace {

constexpr int QB = 64;      // max band width
constexpr int QR = 128;     // rows of a block (2b - 1 padded)
constexpr int NC = 32;      // Z columns per workgroup
constexpr int LV = QB + 1;  // LDS leading dimensions
constexpr int LZ = QR + 1;
constexpr int LW = QB + 1;

__device__ inline int64_t ntasks(int64_t n, int b, int64_t i) { return 1 + (n - 3 - i) / b; }

// Block (g, j): explicit staircase V (written as Vt[s + r*LV], the apply
// kernel's LDS layout) and its forward T factor (T[t + jj*LV]); one
// workgroup of 64 threads per block.
constexpr int LQ = QR + 1;
constexpr int64_t VBLK = (int64_t)QR * LV;  // doubles per packed V block
constexpr int64_t TBLK = (int64_t)QB * LV;  // doubles per packed T block

template <class OT>
__global__ __launch_bounds__(64) void q2_prep_kernel(int64_t n, int b, const double* __restrict__ V2,
                                                     const double* __restrict__ tau2, int64_t maxt, int64_t g,
                                                     OT* VB, OT* TB) {
    __shared__ double Vb[QB * LQ];  // Vb[s*LQ + r]
    __shared__ double Gs[QB * LV];
    __shared__ double Ts[QB * LV];
    __shared__ double y[QB], tv[QB];
    const int t = threadIdx.x;
    const int64_t j = blockIdx.x;
    const int64_t nsw = n - 2;
    const int64_t base = g + 1 + j * b;
    // reflector s of the block is sweep g+s, task j (if it exists)
    {
        const int s = t;
        bool ex = (s < b) && (g + s < nsw) && (j < ntasks(n, b, g + s));
        int L = 0;
        if (ex) {
            int64_t r0 = base + s;
            L = (int)((n - r0) < b ? (n - r0) : b);
        }
        const double* src = V2 + ((g + s) * maxt + j) * (int64_t)b;
        for (int r = 0; r < QR; ++r) {
            int rr = r - s;
            Vb[s * LQ + r] = (ex && rr >= 0 && rr < L) ? src[rr] : 0.0;
        }
        tv[s] = ex ? tau2[(g + s) * maxt + j] : 0.0;
    }
    __syncthreads();
    // Gram G[s1][s2] = sum_r V[r][s1] V[r][s2], thread t = column s2
    for (int s1 = 0; s1 < QB; ++s1) {
        double acc = 0.0;
        for (int r = 0; r < QR; ++r) acc += Vb[s1 * LQ + r] * Vb[t * LQ + r];
        Gs[s1 + t * LV] = acc;
    }
    __syncthreads();
    for (int jj = 0; jj < QB; ++jj) {
        if (t < jj) y[t] = Gs[t + jj * LV];
        __syncthreads();
        if (t < jj) {
            double acc = 0.0;
            for (int k = t; k < jj; ++k) acc += Ts[t + k * LV] * y[k];
            Ts[t + jj * LV] = -tv[jj] * acc;
        }
        if (t == jj) Ts[jj + jj * LV] = tv[jj];
        if (t > jj) Ts[t + jj * LV] = 0.0;
        __syncthreads();
    }
    OT* vout = VB + j * VBLK;
    for (int e = t; e < QR * QB; e += 64) {
        int sidx = e % QB, r = e / QB;
        vout[sidx + r * LV] = (OT)Vb[sidx * LQ + r];
    }
    OT* tout = TB + j * TBLK;
    for (int e = t; e < QB * QB; e += 64) {
        int tt = e % QB, jj = e / QB;
        tout[tt + jj * LV] = (OT)Ts[tt + jj * LV];
    }
}

// Apply the blocks of group g (j ascending) to Z[:, slab].
template <class T>
__global__ __launch_bounds__(256) void q2_apply_kernel(int64_t n, int b, int64_t g, const T* __restrict__ VB,
                                                       const T* __restrict__ TB, T* Z, int64_t ldz, int64_t ncols) {
    typedef fl_tile::Mfma<T> MM;
    typedef typename MM::acc acc_t;
    __shared__ __attribute__((aligned(16))) T Vt[QR * LV];  // Vt[s + r*LV] = V[r][s]
    __shared__ __attribute__((aligned(16))) T Ts[QB * LV];
    __shared__ T Zs[NC * LZ];  // Zs[r + c*LZ]
    __shared__ T W[NC * LW];   // W[s + c*LW]
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int lr = lane >> 4, lc = lane & 15;
    const int64_t col0 = (int64_t)blockIdx.x * NC;
    const int64_t ntg = ntasks(n, b, g);
    for (int64_t j = 0; j < ntg; ++j) {
        const int64_t base = g + 1 + j * b;
        const int rows = (int)((n - base) < QR ? (n - base) : QR);
        // stage the packed V (transposed) and T blocks, and the Z slab
        {
            // 16-byte copies (VBLK and TBLK are multiples of 4 elements; blocks 16-byte aligned)
            const uint4* vsrc = reinterpret_cast<const uint4*>(VB + j * VBLK);
            uint4* vdst = reinterpret_cast<uint4*>(Vt);
            for (int e = t; e < (int)(VBLK * sizeof(T) / 16); e += 256) vdst[e] = vsrc[e];
            const uint4* tsrc = reinterpret_cast<const uint4*>(TB + j * TBLK);
            uint4* tdst = reinterpret_cast<uint4*>(Ts);
            for (int e = t; e < (int)(TBLK * sizeof(T) / 16); e += 256) tdst[e] = tsrc[e];
        }
        for (int e = t; e < QR * NC; e += 256) {
            int r = e % QR, c = e / QR;
            Zs[r + c * LZ] = (r < rows && col0 + c < ncols) ? Z[(base + r) + (col0 + c) * ldz] : T(0);
        }
        __syncthreads();
        // W = V^T Zs  (64 x 32): wave w -> tiles (ti = w, tj = 0, 1)
        {
            acc_t acc[2];
            acc[0] = acc_t{0, 0, 0, 0};
            acc[1] = acc_t{0, 0, 0, 0};
            const int ti = wave;
            for (int k0 = 0; k0 < QR; k0 += 4) {
                T a = Vt[(ti * 16 + lc) + (k0 + lr) * LV];
#pragma unroll
                for (int tj = 0; tj < 2; ++tj) {
                    T bb = Zs[(k0 + lr) + (tj * 16 + lc) * LZ];
                    acc[tj] = MM::mma(a, bb, acc[tj]);
                }
            }
#pragma unroll
            for (int tj = 0; tj < 2; ++tj)
#pragma unroll
                for (int r = 0; r < 4; ++r) W[(ti * 16 + MM::row(lr, r)) + (tj * 16 + lc) * LW] = acc[tj][r];
        }
        __syncthreads();
        // W := T W  (computed in registers, then written over W)
        {
            acc_t acc[2];
            acc[0] = acc_t{0, 0, 0, 0};
            acc[1] = acc_t{0, 0, 0, 0};
            const int ti = wave;
            for (int k0 = 0; k0 < QB; k0 += 4) {
                T a = Ts[(ti * 16 + lc) + (k0 + lr) * LV];
#pragma unroll
                for (int tj = 0; tj < 2; ++tj) {
                    T bb = W[(k0 + lr) + (tj * 16 + lc) * LW];
                    acc[tj] = MM::mma(a, bb, acc[tj]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int tj = 0; tj < 2; ++tj)
#pragma unroll
                for (int r = 0; r < 4; ++r) W[(ti * 16 + MM::row(lr, r)) + (tj * 16 + lc) * LW] = acc[tj][r];
        }
        __syncthreads();
        // Zs -= V W  (128 x 32): wave w -> tiles ti = 2w, 2w+1; tj = 0, 1
        {
            acc_t acc[2][2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) acc[a][c] = acc_t{0, 0, 0, 0};
            for (int k0 = 0; k0 < QB; k0 += 4) {
                T bb[2];
#pragma unroll
                for (int tj = 0; tj < 2; ++tj) bb[tj] = W[(k0 + lr) + (tj * 16 + lc) * LW];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const int ti = 2 * wave + a;
                    T av = Vt[(k0 + lr) + (ti * 16 + lc) * LV];
#pragma unroll
                    for (int tj = 0; tj < 2; ++tj) acc[a][tj] = MM::mma(av, bb[tj], acc[a][tj]);
                }
            }
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int ti = 2 * wave + a;
#pragma unroll
                for (int tj = 0; tj < 2; ++tj)
#pragma unroll
                    for (int r = 0; r < 4; ++r) Zs[(ti * 16 + MM::row(lr, r)) + (tj * 16 + lc) * LZ] -= acc[a][tj][r];
            }
        }
        __syncthreads();
        for (int e = t; e < QR * NC; e += 256) {
            int r = e % QR, c = e / QR;
            if (r < rows && col0 + c < ncols) Z[(base + r) + (col0 + c) * ldz] = Zs[r + c * LZ];
        }
        __syncthreads();
    }
}

}  // namespace
int64_t fl_sy2sb_panels(int64_t n, int b);
namespace {

template <class T>
hipError_t q2_apply_t(hipStream_t s, int64_t n, int b, const double* V2, const double* tau2, int64_t maxt, T* work,
                      T* Z, int64_t ldz, int64_t ncols) {
    static_assert((VBLK * sizeof(float)) % 16 == 0 && (TBLK * sizeof(float)) % 16 == 0, "16-byte blocks");
    if (n < 3 || b < 2) return hipSuccess;
    const int64_t nsw = n - 2;
    T* VB = work;
    T* TB = work + maxt * VBLK;
    hipError_t e;
    const int64_t ngroups = FL_DIV_UP(nsw, b);
    for (int64_t gi = ngroups - 1; gi >= 0; --gi) {
        const int64_t g = gi * b;
        const int64_t nt = 1 + (n - 3 - g) / b;
        q2_prep_kernel<T><<<(unsigned)nt, 64, 0, s>>>(n, b, V2, tau2, maxt, g, VB, TB);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        {
            KScope ks("q2_apply", s);
            q2_apply_kernel<T><<<(unsigned)FL_DIV_UP(ncols, NC), 256, 0, s>>>(n, b, g, VB, TB, Z, ldz, ncols);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class T>
hipError_t q1_apply_t(hipStream_t s, int64_t n, int b, const T* V1, int64_t ldv, const T* T1, T* Z, int64_t ldz,
                      int64_t ncols, T* work) {
    int64_t np = fl_sy2sb_panels(n, b);
    hipError_t e;
    for (int64_t p = np - 1; p >= 0; --p) {
        const int64_t c0 = p * b, r0 = c0 + b, m = n - r0;
        const int kref = (int)std::min<int64_t>(b, m - 1);
        if (kref <= 0) continue;
        const T* Vp = V1 + r0 + c0 * ldv;
        const T* Tp = T1 + p * (int64_t)b * b;
        T* W1 = work;
        T* W2 = work + (int64_t)b * ncols;
        if ((e = fl_gemm_t(s, 1, 0, kref, ncols, m, 1.0, Vp, ldv, Z + r0, ldz, 0.0, W1, b))) return e;
        if ((e = fl_gemm_t(s, 0, 0, kref, ncols, kref, 1.0, Tp, b, W1, b, 0.0, W2, b))) return e;
        if ((e = fl_gemm_t(s, 0, 0, m, ncols, kref, -1.0, Vp, ldv, W2, b, 1.0, Z + r0, ldz))) return e;
    }
    return hipSuccess;
}

}  // namespace

// Packed blocks of one group: maxt V blocks and maxt T blocks (elements).
int64_t fl_q2_t_elems(int64_t n, int b, int64_t maxt) { (void)n; (void)b; return maxt * (VBLK + TBLK) + 4; }

// Z (n x ncols) := Q2 Z with the reflectors of fl_sb2st.  work: fl_q2_t_elems elements.
hipError_t fl_q2_apply(hipStream_t s, int64_t n, int b, const double* V2, const double* tau2, int64_t maxt, double* work,
                       double* Z, int64_t ldz, int64_t ncols) {
    return q2_apply_t<double>(s, n, b, V2, tau2, maxt, work, Z, ldz, ncols);
}
hipError_t fl_q2_apply_f(hipStream_t s, int64_t n, int b, const double* V2, const double* tau2, int64_t maxt,
                         float* work, float* Z, int64_t ldz, int64_t ncols) {
    return q2_apply_t<float>(s, n, b, V2, tau2, maxt, work, Z, ldz, ncols);
}

// Z (n x ncols) := Q1 Z, Q1 = prod over panels of (I - V_p T_p V_p^T).
// work: >= 2 * b * ncols elements.
hipError_t fl_q1_apply(hipStream_t s, int64_t n, int b, const double* V1, int64_t ldv, const double* T1, double* Z,
                       int64_t ldz, int64_t ncols, double* work) {
    return q1_apply_t<double>(s, n, b, V1, ldv, T1, Z, ldz, ncols, work);
}
hipError_t fl_q1_apply_f(hipStream_t s, int64_t n, int b, const float* V1, int64_t ldv, const float* T1, float* Z,
                         int64_t ldz, int64_t ncols, float* work) {
    return q1_apply_t<float>(s, n, b, V1, ldv, T1, Z, ldz, ncols, work);
}
