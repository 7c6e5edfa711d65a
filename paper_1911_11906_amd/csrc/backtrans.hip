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

// ---- band width 64: one launch, Z windows resident in registers ----------
//
// Block (g, j) is viewed in a 128-row frame starting at row g + 64 j (one row
// above its first reflector row), so that consecutive blocks of a group move
// by exactly half a frame and every frame starts on a 64-row boundary.  In
// frame coordinates reflector s has its entries at rows s+1 .. s+64, so V is
// nonzero only on 16 x 16 tile pairs (frame tile rt, reflector tile wt) with
// wt <= rt <= wt + 4, and T is upper triangular; products over the other
// tile pairs are skipped.
//
// A workgroup owns 64 columns of Z, a wave 16 of them.  Each wave holds the
// current 128 x 16 window of its columns in MFMA accumulator registers:
// lane (lr, lc), register r of frame tile rt is row 16 rt + 4 lr + r of
// column lc.  That layout is at the same time the B-operand layout of
// W = V^T Z (any order of the reduction index is allowed, and V is read from
// LDS to match it) and, up to a permutation inside each 16-row tile, the
// output layout of Z -= V (T W).  After a block the upper half of the window
// is final for the group and goes to memory; the lower half becomes the
// upper half of the next block.  V of the next block (a contiguous 64 x 64
// chunk written beside its T factor) and the T factor are fetched into
// registers while the current block computes.
constexpr int FB = 64;       // band width of this path
constexpr int FR = 2 * FB;   // frame rows
constexpr int LDF = FB + 4;  // LDS stride of the V frame (spreads banks for both read patterns)

__host__ __device__ inline int64_t q2_block_base(int64_t gi, int64_t n0) { return gi * n0 - gi * (gi - 1) / 2; }

// Workgroup barrier that orders LDS only.  Every entry of Z is loaded and
// stored by one and the same lane (its column fixes the wave, its row modulo
// 16 the lane), so the waves share nothing through global memory and need
// not wait for their stores to land: those drain while the next block runs.
__device__ inline void q2_lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Frame-row offset, inside a 16-row tile, of MFMA output index p when lane
// (lr, lc) register r holds row 4 lr + r.
template <class T> __device__ inline int q2_sigma(int p);
template <> __device__ inline int q2_sigma<double>(int p) { return 4 * (p & 3) + (p >> 2); }  // p = lr + 4 r
template <> __device__ inline int q2_sigma<float>(int p) { return p; }                        // p = 4 lr + r

// Forward T factor of every block (g = 64 gi, j): T upper triangular with
// H(g, j) ... H(g+63, j) = I - V T V^T.  T[t][jj] = -tau_jj sum_k T[t][k] G[k][jj]
// over t <= k < jj, with G = V^T V.  Output column-major 64 x 64 per block,
// blocks of group gi from q2_block_base(gi, n0).  The block's reflectors go
// to VB in the same order, 64 x 64 per block (VB[64 s + i]: entry i of
// reflector s, zero where the reflector or the entry does not exist), so
// that the application reads one contiguous, unmasked chunk per block.
template <class OT>
__global__ __launch_bounds__(256) void q2_tfactor_kernel(int64_t n, int64_t maxt, int64_t n0,
                                                         const double* __restrict__ V2,
                                                         const double* __restrict__ tau2, OT* __restrict__ TB,
                                                         OT* __restrict__ VB) {
    const int64_t gi = blockIdx.y, j = blockIdx.x;
    if (j >= n0 - gi) return;
    constexpr int LC = FB + 1;
    __shared__ double Vc[FB * LC];  // Vc[s*LC + i]: entry i of reflector s
    __shared__ double Gs[FB * LC];  // Gs[k + jj*LC] = G[k][jj], k < jj
    __shared__ double tv[FB];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t g = gi * FB, nsw = n - 2;
    for (int s = wave; s < FB; s += 4) {
        const int64_t sw = g + s;
        const bool ex = sw < nsw && j < 1 + (n - 3 - sw) / FB;
        const int64_t r0 = g + 1 + j * FB + s;
        const int L = ex ? (int)((n - r0) < FB ? (n - r0) : FB) : 0;
        Vc[s * LC + lane] = lane < L ? V2[(sw * maxt + j) * FB + lane] : 0.0;
        if (lane == 0) tv[s] = ex ? tau2[sw * maxt + j] : 0.0;
    }
    __syncthreads();
    {
        OT* vb = VB + (q2_block_base(gi, n0) + j) * (int64_t)(FB * FB);
        for (int s = wave; s < FB; s += 4) vb[s * FB + lane] = (OT)Vc[s * LC + lane];
    }
    // G[k][jj] (k < jj): rows s.t. both reflectors are nonzero; thread -> (jj, k mod 4)
    {
        const int jj = lane, q = wave;
        for (int k = q; k < FB - 1; k += 4) {
            if (k < jj) {
                const int d = jj - k, len = FB - d;
                double acc = 0.0;
                for (int i = 0; i < len; ++i) acc += Vc[k * LC + i + d] * Vc[jj * LC + i];
                Gs[k + jj * LC] = acc;
            }
        }
    }
    __syncthreads();
    if (wave != 0) return;
    double Tr[FB];  // row t of T
#pragma unroll
    for (int k = 0; k < FB; ++k) Tr[k] = 0.0;
#pragma unroll
    for (int jj = 0; jj < FB; ++jj) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < jj; ++k) acc += Tr[k] * Gs[k + jj * LC];  // Tr[k] = 0 for k < t
        const double tau = tv[jj];
        Tr[jj] = lane < jj ? -tau * acc : (lane == jj ? tau : 0.0);
    }
    OT* out = TB + (q2_block_base(gi, n0) + j) * (int64_t)(FB * FB);
#pragma unroll
    for (int k = 0; k < FB; ++k) out[lane + k * FB] = (OT)Tr[k];
}

// Rows row0 .. row0+3 of column zc.  Loads are unconditional: with CLAMP
// (a window reaching past row n-1) the indices are clamped into the matrix,
// so rows at or beyond n hold copies of row n-1, which is harmless since V
// is zero there and those rows are never stored.
template <class T, bool VEC, bool CLAMP>
__device__ inline void q2_load4(const T* zc, int64_t row0, int64_t n, typename fl_tile::Mfma<T>::acc& a) {
    if (CLAMP) {
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = zc[row0 + r < n ? row0 + r : n - 1];
    } else if (VEC) {
        if constexpr (sizeof(T) == 4) {
            const float4 v = *reinterpret_cast<const float4*>(zc + row0);
            a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
        } else {
            const double2 v0 = *reinterpret_cast<const double2*>(zc + row0);
            const double2 v1 = *reinterpret_cast<const double2*>(zc + row0 + 2);
            a[0] = v0.x; a[1] = v0.y; a[2] = v1.x; a[3] = v1.y;
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = zc[row0 + r];
    }
}

template <class T, bool VEC, bool MASK>
__device__ inline void q2_store4(T* zc, int64_t row0, int64_t n, bool cok, const typename fl_tile::Mfma<T>::acc& a) {
    if (!cok) return;
    if (MASK) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (row0 + r < n) zc[row0 + r] = a[r];
    } else if (VEC) {
        if constexpr (sizeof(T) == 4) {
            *reinterpret_cast<float4*>(zc + row0) = make_float4(a[0], a[1], a[2], a[3]);
        } else {
            *reinterpret_cast<double2*>(zc + row0) = make_double2(a[0], a[1]);
            *reinterpret_cast<double2*>(zc + row0 + 2) = make_double2(a[2], a[3]);
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) zc[row0 + r] = a[r];
    }
}

template <class T, bool VEC>
__global__ __launch_bounds__(256) void q2_apply64_kernel(int64_t n, int64_t n0, const T* __restrict__ VB,
                                                         const T* __restrict__ TB, T* __restrict__ Z, int64_t ldz,
                                                         int64_t ncols) {
    typedef fl_tile::Mfma<T> MM;
    typedef typename MM::acc acc_t;
    // The four A operands of one lane in one 16 x 16 tile pair (r = 0..3)
    // are contiguous in LDS, read as 16-byte groups that are conflict-free
    // over each 16 lanes.  FP32: V twice (row-major Vf for Z -= V W2,
    // reflector-major VW for W = V^T Z) and T transposed.  FP64 (whose MFMA
    // output row of lane (lr, r) is lr + 4 r, not 4 lr + r): row-major Vf and
    // transposed T with the columns of every 16-wide tile permuted by
    // pcol, so that logical column lr + 4 r sits at 4 lr + r; W = V^T Z
    // reads single values (row stride 132 words: at most two lanes per
    // bank).
    constexpr bool F32 = sizeof(T) == 4;
    constexpr int LDW = FR + 4;                // VW stride (frame rows + 4)
    constexpr int LDV = F32 ? LDF : FB + 2;    // Vf stride
    constexpr int LDT = FB + (F32 ? 4 : 2);    // Ts stride
    __shared__ __attribute__((aligned(16))) T Vf[FR * LDV];                // Vf[k*LDV + pcol(s)] = V[k][s], frame row k
    __shared__ __attribute__((aligned(16))) T VW[F32 ? FB * LDW : 1];     // VW[s*LDW + k] = V[k][s]
    __shared__ __attribute__((aligned(16))) T Ts[FB * LDT];               // Ts[i*LDT + pcol(k)] = T[i][k]
    auto pcol = [](int c) { return F32 ? c : (c & ~15) | (4 * (c & 3) + ((c >> 2) & 3)); };
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int lr = lane >> 4, lc = lane & 15;
    const int64_t col = (int64_t)blockIdx.x * 64 + wave * 16 + lc;
    const bool cok = col < ncols;
    T* zc = Z + (cok ? col : 0) * ldz;
    for (int e = t; e < FR * LDV; e += 256) Vf[e] = T(0);  // off-staircase entries stay zero
    if constexpr (F32)
        for (int e = t; e < FB * LDW; e += 256) VW[e] = T(0);

    T pv[16], pt[16];
    // block (g, j): element t + 256 q of its V chunk is entry i = lane of
    // reflector s = wave + 4 q, at frame row s + 1 + i.
    auto fetch = [&](int64_t gi, int64_t j) {
        const int64_t off = (q2_block_base(gi, n0) + j) * (int64_t)(FB * FB);
#pragma unroll
        for (int q = 0; q < 16; ++q) pv[q] = VB[off + t + 256 * q];
#pragma unroll
        for (int q = 0; q < 16; ++q) pt[q] = TB[off + t + 256 * q];
    };
    auto stage = [&]() {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int s = wave + 4 * q;
            Vf[(s + 1 + lane) * LDV + pcol(s)] = pv[q];
            if constexpr (F32) VW[s * LDW + s + 1 + lane] = pv[q];
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int e = t + 256 * q;
            Ts[(e & (FB - 1)) * LDT + pcol(e / FB)] = pt[q];
        }
    };

    const int lrow = 4 * lr;
    const int vsig = q2_sigma<T>(lc);
    acc_t zt[4], zb[4], zn[4];
    // One block on the window (zt, zb): products, zt to memory, then the
    // window moves down by half; the lower half of the next window is loaded
    // into zn meanwhile.  TAIL: the window or the rows loaded reach past n-1.
    auto block = [&](auto tail, int64_t gi, int64_t j, int64_t nt) {
        constexpr bool TAIL = decltype(tail)::value;
        const int64_t F = gi * FB + j * FB;
        const bool more = j + 1 < nt;
        if (more) {
            fetch(gi, j + 1);
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) q2_load4<T, VEC, TAIL>(zc, F + 2 * FB + 16 * rt + lrow, n, zn[rt]);
        }
        acc_t w[4], w2[4];
        // W = V^T Z over tile pairs wt <= rt <= wt + 4
#pragma unroll
        for (int wt = 0; wt < 4; ++wt) w[wt] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int d = 0; d < 5; ++d) {
            T a[4][4];  // a[wt][r]
#pragma unroll
            for (int wt = 0; wt < 4; ++wt) {
                const int rt = wt + d;
                if constexpr (F32) {
                    const float4 v = *reinterpret_cast<const float4*>(&VW[(16 * wt + lc) * LDW + 16 * rt + lrow]);
                    a[wt][0] = v.x; a[wt][1] = v.y; a[wt][2] = v.z; a[wt][3] = v.w;
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) a[wt][r] = Vf[(16 * rt + lrow + r) * LDV + 16 * wt + pcol(lc)];
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int wt = 0; wt < 4; ++wt) {
                    const int rt = wt + d;
                    const T bz = rt < 4 ? zt[rt & 3][r] : zb[rt & 3][r];
                    w[wt] = MM::mma(a[wt][r], bz, w[wt]);
                }
        }
        // W2 = T W (T upper triangular)
#pragma unroll
        for (int wt = 0; wt < 4; ++wt) w2[wt] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            T a[4][4];  // a[wt2][r]
#pragma unroll
            for (int wt2 = 0; wt2 + d < 4; ++wt2) {
                const int wt = wt2 + d;
                const T* src = &Ts[(16 * wt2 + lc) * LDT + 16 * wt + lrow];  // column pcol(16 wt + row(lr, r))
                if constexpr (F32) {
                    const float4 v = *reinterpret_cast<const float4*>(src);
                    a[wt2][0] = v.x; a[wt2][1] = v.y; a[wt2][2] = v.z; a[wt2][3] = v.w;
                } else {
                    const double2 v0 = *reinterpret_cast<const double2*>(src);
                    const double2 v1 = *reinterpret_cast<const double2*>(src + 2);
                    a[wt2][0] = v0.x; a[wt2][1] = v0.y; a[wt2][2] = v1.x; a[wt2][3] = v1.y;
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int wt2 = 0; wt2 + d < 4; ++wt2) w2[wt2] = MM::mma(a[wt2][r], w[wt2 + d][r], w2[wt2]);
        }
#pragma unroll
        for (int wt = 0; wt < 4; ++wt)
#pragma unroll
            for (int r = 0; r < 4; ++r) w2[wt][r] = -w2[wt][r];
        // Z -= V W2
#pragma unroll
        for (int d = 0; d < 5; ++d) {
            T a[4][4];  // a[wt][r]
#pragma unroll
            for (int wt = 0; wt < 4; ++wt) {
                const int rt = wt + d;
                const T* src = &Vf[(16 * rt + vsig) * LDV + 16 * wt + lrow];  // column pcol(16 wt + row(lr, r))
                if constexpr (F32) {
                    const float4 v = *reinterpret_cast<const float4*>(src);
                    a[wt][0] = v.x; a[wt][1] = v.y; a[wt][2] = v.z; a[wt][3] = v.w;
                } else {
                    const double2 v0 = *reinterpret_cast<const double2*>(src);
                    const double2 v1 = *reinterpret_cast<const double2*>(src + 2);
                    a[wt][0] = v0.x; a[wt][1] = v0.y; a[wt][2] = v1.x; a[wt][3] = v1.y;
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int wt = 0; wt < 4; ++wt) {
                    const int rt = wt + d;
                    if (rt < 4)
                        zt[rt & 3] = MM::mma(a[wt][r], w2[wt][r], zt[rt & 3]);
                    else
                        zb[rt & 3] = MM::mma(a[wt][r], w2[wt][r], zb[rt & 3]);
                }
        }
        if (more) {
            // keep the prefetched rows out of the products: without this
            // ordering point the compiler may move the copy into zb (and the
            // wait for those loads) in among the matrix instructions.  It
            // sits before the stores below, so that the wait for the loads
            // cannot turn into a wait for the stores as well, and it takes
            // the last product of every tile, so that it cannot be scheduled
            // (with its wait) before the final product of any of them.
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    asm volatile("" : "+v"(zn[rt][r])
                                 : "v"(zt[0][3]), "v"(zt[1][3]), "v"(zt[2][3]), "v"(zt[3][3]),
                                   "v"(zb[0][3]), "v"(zb[1][3]), "v"(zb[2][3]), "v"(zb[3][3]));
        }
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) q2_store4<T, VEC, TAIL>(zc, F + 16 * rt + lrow, n, cok, zt[rt]);
        asm volatile("" ::: "memory");  // issue the stores here, before the staging keeps zt live
        if (more) {
            q2_lds_barrier();  // every wave is done with this block's V and T
            stage();
            q2_lds_barrier();
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                zt[rt] = zb[rt];
                zb[rt] = zn[rt];
            }
        } else {
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) q2_store4<T, VEC, true>(zc, F + FB + 16 * rt + lrow, n, cok, zb[rt]);
        }
    };

    for (int64_t gi = n0 - 1; gi >= 0; --gi) {
        const int64_t g = gi * FB, nt = n0 - gi;
        fetch(gi, 0);
        q2_lds_barrier();  // the previous group's last block is done with the LDS
        stage();
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            q2_load4<T, VEC, true>(zc, g + 16 * rt + lrow, n, zt[rt]);
            q2_load4<T, VEC, true>(zc, g + FB + 16 * rt + lrow, n, zb[rt]);
        }
        // wait for the window loads here: a wait for them carried into the
        // blocks would, in every block, stall the products until that
        // block's prefetch has landed
        __builtin_amdgcn_s_waitcnt(0);
        q2_lds_barrier();
        // blocks whose window and prefetched rows lie inside the matrix
        const int64_t nfull = n - g >= 3 * FB ? (n - g - 3 * FB) / FB + 1 : 0;
        int64_t j = 0;
        for (; j < nt && j < nfull; ++j) block(std::false_type{}, gi, j, nt);
        for (; j < nt; ++j) block(std::true_type{}, gi, j, nt);
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
    if (b == FB) {
        const int64_t n0 = 1 + (n - 3) / FB;  // groups, and tasks of the first sweep of group 0
        T* VB = work + q2_block_base(n0, n0) * FB * FB;
        q2_tfactor_kernel<T><<<dim3((unsigned)n0, (unsigned)n0), 256, 0, s>>>(n, maxt, n0, V2, tau2, work, VB);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const bool vec = (reinterpret_cast<uintptr_t>(Z) % 16 == 0) && ((ldz * (int64_t)sizeof(T)) % 16 == 0);
        const unsigned grid = (unsigned)FL_DIV_UP(ncols, 64);
        KScope ks("q2_apply", s);
        if (vec)
            q2_apply64_kernel<T, true><<<grid, 256, 0, s>>>(n, n0, VB, work, Z, ldz, ncols);
        else
            q2_apply64_kernel<T, false><<<grid, 256, 0, s>>>(n, n0, VB, work, Z, ldz, ncols);
        return hipGetLastError();
    }
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

// Q1 = H_0 H_1 ... H_{np-1}, H_p = I - V_p T_p V_p^T.  QG consecutive panels
// are merged into one block reflector (their V columns are adjacent in V1,
// and the rows of a later panel above its own first row are zero), with
//   T = [T_a  -T_a (V_a^T V_b) T_b; 0  T_b]
// built panel by panel, so that each group costs three GEMMs with inner or
// outer dimension QG b instead of b.  Groups are applied last first.
constexpr int QG = 8;

template <class T>
hipError_t q1_apply_t(hipStream_t s, int64_t n, int b, const T* V1, int64_t ldv, const T* T1, T* Z, int64_t ldz,
                      int64_t ncols, T* work) {
    const int64_t np = fl_sy2sb_panels(n, b);
    const int64_t KM = (int64_t)QG * b;
    T* Gr = work;          // KM x KM: V^T V of the group
    T* Tg = Gr + KM * KM;  // KM x KM: merged T
    T* Yb = Tg + KM * KM;  // KM x b
    T* W1 = Yb + KM * b;   // KM x ncols
    T* W2 = W1 + KM * ncols;
    hipError_t e;
    auto kref_of = [&](int64_t p) { return (int)std::min<int64_t>(b, n - (p * b + b) - 1); };
    for (int64_t gi = FL_DIV_UP(np, QG) - 1; gi >= 0; --gi) {
        const int64_t p0 = gi * QG, p1 = std::min<int64_t>(np, p0 + QG);
        const int64_t c0 = p0 * b, r0 = c0 + b, m = n - r0;
        int64_t K = 0;
        for (int64_t p = p0; p < p1; ++p) K += kref_of(p);
        if (K <= 0) continue;
        const T* V = V1 + r0 + c0 * ldv;
        const T* Tm = T1 + p0 * (int64_t)b * b;
        int64_t ldt = b;
        if (p1 - p0 > 1) {
            if ((e = fl_gemm_t(s, 1, 0, K, K, m, 1.0, V, ldv, V, ldv, 0.0, Gr, KM))) return e;
            if ((e = hipMemsetAsync(Tg, 0, sizeof(T) * KM * KM, s))) return e;
            int64_t off = 0;
            for (int64_t p = p0; p < p1; ++p) {
                const int kq = kref_of(p);
                if ((e = hipMemcpy2DAsync(Tg + off + off * KM, sizeof(T) * KM, T1 + p * (int64_t)b * b, sizeof(T) * b,
                                          sizeof(T) * kq, kq, hipMemcpyDeviceToDevice, s)))
                    return e;
                if (off > 0) {
                    // Tg[0:off, off:off+kq] = -Tg[0:off, 0:off] (V_a^T V_b) T_b
                    if ((e = fl_gemm_t(s, 0, 0, off, kq, off, 1.0, Tg, KM, Gr + off * KM, KM, 0.0, Yb, KM))) return e;
                    if ((e = fl_gemm_t(s, 0, 0, off, kq, kq, -1.0, Yb, KM, Tg + off + off * KM, KM, 0.0, Tg + off * KM,
                                       KM)))
                        return e;
                }
                off += kq;
            }
            Tm = Tg;
            ldt = KM;
        }
        if ((e = fl_gemm_t(s, 1, 0, K, ncols, m, 1.0, V, ldv, Z + r0, ldz, 0.0, W1, KM))) return e;
        if ((e = fl_gemm_t(s, 0, 0, K, ncols, K, 1.0, Tm, ldt, W1, KM, 0.0, W2, KM))) return e;
        if ((e = fl_gemm_t(s, 0, 0, m, ncols, K, -1.0, V, ldv, W2, KM, 1.0, Z + r0, ldz))) return e;
    }
    return hipSuccess;
}

}  // namespace

// Work elements: with b = 64 the T factors of every block, otherwise the
// packed V and T blocks of one group.
int64_t fl_q2_t_elems(int64_t n, int b, int64_t maxt) {
    if (b == FB && n >= 3) {
        const int64_t n0 = 1 + (n - 3) / FB;
        return 2 * q2_block_base(n0, n0) * FB * FB + 4;  // T factors and reflectors of every block
    }
    return maxt * (VBLK + TBLK) + 4;
}

// Z (n x ncols) := Q2 Z with the reflectors of fl_sb2st.  work: fl_q2_t_elems elements.
hipError_t fl_q2_apply(hipStream_t s, int64_t n, int b, const double* V2, const double* tau2, int64_t maxt, double* work,
                       double* Z, int64_t ldz, int64_t ncols) {
    return q2_apply_t<double>(s, n, b, V2, tau2, maxt, work, Z, ldz, ncols);
}
hipError_t fl_q2_apply_f(hipStream_t s, int64_t n, int b, const double* V2, const double* tau2, int64_t maxt,
                         float* work, float* Z, int64_t ldz, int64_t ncols) {
    return q2_apply_t<float>(s, n, b, V2, tau2, maxt, work, Z, ldz, ncols);
}

// Work elements of fl_q1_apply for ncols columns.
int64_t fl_q1_work_elems(int64_t n, int b, int64_t ncols) {
    (void)n;
    const int64_t KM = (int64_t)QG * b;
    return 2 * KM * KM + KM * b + 2 * KM * ncols;
}

// Z (n x ncols) := Q1 Z, Q1 = prod over panels of (I - V_p T_p V_p^T).  V1
// must be zero above each panel's first reflector row.  work:
// fl_q1_work_elems(n, b, ncols) elements.
hipError_t fl_q1_apply(hipStream_t s, int64_t n, int b, const double* V1, int64_t ldv, const double* T1, double* Z,
                       int64_t ldz, int64_t ncols, double* work) {
    return q1_apply_t<double>(s, n, b, V1, ldv, T1, Z, ldz, ncols, work);
}
hipError_t fl_q1_apply_f(hipStream_t s, int64_t n, int b, const float* V1, int64_t ldv, const float* T1, float* Z,
                         int64_t ldz, int64_t ncols, float* work) {
    return q1_apply_t<float>(s, n, b, V1, ldv, T1, Z, ldz, ncols, work);
}
