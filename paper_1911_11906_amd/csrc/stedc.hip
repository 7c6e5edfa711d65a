// Symmetric tridiagonal eigensolver: Cuppen's divide and conquer.
//
// T = diag(T1, T2) + rho u u^T with u = e_m + sign(beta) e_{m+1}, rho = |beta|
// (beta the coupling entry); the last diagonal entry of T1 and the first of T2
// are reduced by rho.  Given T1 = Q1 D1 Q1^T, T2 = Q2 D2 Q2^T, the merged
// problem is D + rho' z z^T with z = Q^T u / sqrt(2), rho' = 2 rho.
//  * deflation: rho'|z_j| <= tol, or two close poles made to share one z by a
//    Givens rotation whose off-diagonal residue is <= tol;
//  * each remaining root lambda_k of 1 + rho' sum z_j^2/(d_j - lambda) = 0 is
//    found by one thread in coordinates shifted to its nearer pole (a
//    two-pole rational model with a bisection safeguard), keeping
//    d_j - lambda_k to full relative accuracy;
//  * z is recomputed from the roots (Gu and Eisenstat) so that the vectors
//    zhat_j / (d_j - lambda_k) are numerically orthogonal;
//  * the merged eigenvectors are Q times those vectors: two GEMMs on the
//    matrix cores, exploiting the block structure of Q (columns that live only
//    in the top or only in the bottom half).
// The leaves (<= 64) use implicit QL with Wilkinson shifts, one workgroup per
// leaf.  All merges of one tree level run in the same launches; nothing
// returns to the host between levels.
#include <algorithm>
#include <cfloat>
#include <vector>
#include "internal.h"

namespace {

constexpr int LEAF_MAX = 64;
constexpr double EPS = DBL_EPSILON;

struct MergeDesc {
    int64_t o;   // first row/column of the merged block
    int64_t N;   // size
    int64_t n1;  // size of the first child
};

// per-merge counters written on the device
struct MergeCounts {
    int64_t K;      // non-deflated
    int64_t ndefl;  // deflated
    int64_t nrot;   // Givens rotations
    int64_t c1, c2, c3;  // kept columns by type (top only / both / bottom only)
    double rho2;
};

// ------------------------------------------------------------------ leaves
__global__ __launch_bounds__(64) void leaf_kernel(const int64_t* __restrict__ leaf_lo, const int* __restrict__ leaf_m,
                                                  double* d, const double* __restrict__ e, double* Z, int64_t ldz,
                                                  int* fail) {
    __shared__ double zs[LEAF_MAX * LEAF_MAX];  // column-major, ld LEAF_MAX
    __shared__ double dd[LEAF_MAX], ee[LEAF_MAX];
    __shared__ double rc[LEAF_MAX], rs[LEAF_MAX];
    __shared__ int rlo, rhi, go;
    const int t = threadIdx.x;
    const int64_t lo = leaf_lo[blockIdx.x];
    const int m = leaf_m[blockIdx.x];
    for (int c = 0; c < m; ++c) zs[t + c * LEAF_MAX] = (t == c) ? 1.0 : 0.0;
    if (t < m) dd[t] = d[lo + t];
    if (t < m) ee[t] = (t < m - 1) ? e[lo + t] : 0.0;
    __syncthreads();
    for (int l = 0; l < m; ++l) {
        int iter = 0;
        while (true) {
            if (t == 0) {
                int mm = l;
                while (mm < m - 1) {
                    if (fabs(ee[mm]) <= EPS * (fabs(dd[mm]) + fabs(dd[mm + 1]))) break;
                    ++mm;
                }
                go = 0;
                if (mm != l) {
                    if (++iter > 90) {
                        *fail = 1;
                    } else {
                        go = 1;
                        double g = (dd[l + 1] - dd[l]) / (2.0 * ee[l]);
                        double r = hypot(g, 1.0);
                        g = dd[mm] - dd[l] + ee[l] / (g + (g >= 0.0 ? r : -r));
                        double s = 1.0, c = 1.0, p = 0.0;
                        int i = mm - 1;
                        bool early = false;
                        for (; i >= l; --i) {
                            double f = s * ee[i], b = c * ee[i];
                            r = hypot(f, g);
                            ee[i + 1] = r;
                            if (r == 0.0) {
                                dd[i + 1] -= p;
                                ee[mm] = 0.0;
                                early = true;
                                break;
                            }
                            s = f / r;
                            c = g / r;
                            g = dd[i + 1] - p;
                            r = (dd[i] - g) * s + 2.0 * c * b;
                            p = s * r;
                            dd[i + 1] = g + p;
                            g = c * r - b;
                            rc[i] = c;
                            rs[i] = s;
                        }
                        // rotations rc/rs[i] for i in (stop, mm-1] were generated, highest first
                        rlo = early ? i + 1 : l;
                        rhi = mm - 1;
                        if (!early) {
                            dd[l] -= p;
                            ee[l] = g;
                            ee[mm] = 0.0;
                        }
                    }
                }
            }
            __syncthreads();
            if (!go) break;
            // apply the rotations in generation order (i from rhi down to rlo) to row t
            if (t < m) {
                for (int i = rhi; i >= rlo; --i) {
                    double c = rc[i], s = rs[i];
                    double f = zs[t + (i + 1) * LEAF_MAX];
                    double a = zs[t + i * LEAF_MAX];
                    zs[t + (i + 1) * LEAF_MAX] = s * a + c * f;
                    zs[t + i * LEAF_MAX] = c * a - s * f;
                }
            }
            __syncthreads();
        }
    }
    if (t < m) d[lo + t] = dd[t];
    for (int c = 0; c < m; ++c)
        if (t < m) Z[(lo + t) + (lo + c) * ldz] = zs[t + c * LEAF_MAX];
}

// d[s] -= |e[s]|, d[s+1] -= |e[s]| for every split point s (sequential: a
// diagonal entry may sit next to two split points).
__global__ void split_adjust_kernel(const int64_t* __restrict__ splits, int ns, double* d, const double* e) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = 0; i < ns; ++i) {
        int64_t s = splits[i];
        double a = fabs(e[s]);
        d[s] -= a;
        d[s + 1] -= a;
    }
}

// ------------------------------------------------------------------ sorting
// rank of item i among vals[0..N) (ties broken by index), LDS tiled.
__device__ inline int64_t rank_of(const double* vals, int64_t N, int64_t i, double vi, double* tile) {
    int64_t r = 0;
    for (int64_t base = 0; base < N; base += 1024) {
        __syncthreads();
        for (int q = threadIdx.x; q < 1024; q += blockDim.x) tile[q] = (base + q < N) ? vals[base + q] : 0.0;
        __syncthreads();
        int64_t lim = (N - base) < 1024 ? (N - base) : 1024;
        if (i < N) {
            for (int64_t q = 0; q < lim; ++q) {
                double v = tile[q];
                int64_t j = base + q;
                r += (v < vi || (v == vi && j < i)) ? 1 : 0;
            }
        }
    }
    return r;
}

// sort the children's eigenvalues; build z (with the 1/sqrt(2) scaling)
__global__ __launch_bounds__(256) void merge_sort_kernel(const MergeDesc* __restrict__ md, const double* __restrict__ D,
                                                         const double* __restrict__ Z, int64_t ldz,
                                                         const double* __restrict__ e, double* ds, double* zsrt,
                                                         int64_t* perm, int* typ) {
    __shared__ double tile[1024];
    const MergeDesc g = md[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((int64_t)blockIdx.x * blockDim.x >= g.N) return;
    const double* Dv = D + g.o;
    double vi = (i < g.N) ? Dv[i] : 0.0;
    int64_t r = rank_of(Dv, g.N, i, vi, tile);
    if (i >= g.N) return;
    const double beta = e[g.o + g.n1 - 1];
    const double sgn = beta >= 0.0 ? 1.0 : -1.0;
    const double inv_sqrt2 = 0.70710678118654752440;
    double zi = (i < g.n1) ? Z[(g.o + g.n1 - 1) + (g.o + i) * ldz] : sgn * Z[(g.o + g.n1) + (g.o + i) * ldz];
    ds[g.o + r] = vi;
    zsrt[g.o + r] = zi * inv_sqrt2;
    perm[g.o + r] = i;
    typ[g.o + i] = (i < g.n1) ? 1 : 3;
}

// Deflation: one workgroup per merge.  The result is that of one scan over
// the sorted poles: a pole with rho' |z| <= tol deflates; among the others,
// a candidate and the next pole whose Givens rotation leaves a residue
// |(d_j - d_c) c s| <= tol are rotated (the candidate deflates, the next
// pole carries z = r and becomes the candidate), else the candidate is kept.
// Only a rotation changes the state that the next test sees, so the scan
// runs in chunks of DCH sorted poles: (1) flags and the list of
// non-deflated poles (prefix sums), (2) every consecutive pair tested in
// parallel with its original values, (3) one thread walks only the pairs
// that rotate and the chains of tests that follow a rotation, (4) the kept
// poles, the deflated ones (in scan order) and the counts are written by
// prefix sums.  The last pole of a chunk is carried into the next one as
// the candidate.  Every value is computed by the same expressions in the
// same order as the one-thread scan, so the results are the same bits.
constexpr int DCH = 2048;          // sorted poles per chunk
constexpr int DNT = 512;           // threads
constexpr int DPT = DCH / DNT;     // chunk positions per thread (contiguous)

struct DeflLds {
    double sd[DCH], sz[DCH];       // chunk poles and z
    int64_t sp[DCH];               // their columns
    int L[DCH];                    // chunk position of non-deflated pole u
    int U[DCH];                    // u of a non-deflated chunk position
    int F[DCH];                    // u whose pair (u-1, u) rotates when both are original
    unsigned char fate[DCH];       // 0 kept (original values), 1 kept (modified), 2 deflated by rotation
    unsigned char hasrot[DCH];     // a rotation deflates u-1 into u
    double kd[DCH], kz[DCH];       // modified values of a kept pole
    double rv[DCH];                // value deflated by the rotation at u
    int64_t rcol[DCH];             // its column
    int64_t sc[DNT];               // scan scratch
    double red[DNT];
    int keptc;                     // the carried candidate was kept at the chunk's start
};

// rotation test of candidate (cd, cz) against pole (dj, zj)
__device__ inline bool defl_rotates(double cd, double cz, double dj, double zj, double tol, double& c, double& sn,
                                    double& r) {
    // |z| <= 1 and, not deflated, rho' |z| > tol: the squares neither
    // overflow nor underflow, so no hypot is needed
    r = sqrt(cz * cz + zj * zj);
    const double ir = 1.0 / r;
    c = zj * ir;
    sn = cz * ir;
    const double tt = dj - cd;
    return fabs(tt * c * sn) <= tol;
}

// exclusive prefix sum of v over the workgroup's threads (in thread order);
// *total receives the sum
__device__ inline int64_t defl_scan(int64_t v, DeflLds& s, int64_t* total) {
    const int t = threadIdx.x;
    __syncthreads();
    s.sc[t] = v;
    __syncthreads();
    for (int o = 1; o < DNT; o <<= 1) {
        const int64_t a = (t >= o) ? s.sc[t - o] : 0;
        __syncthreads();
        s.sc[t] += a;
        __syncthreads();
    }
    *total = s.sc[DNT - 1];
    return s.sc[t] - v;
}

__global__ __launch_bounds__(DNT) void merge_deflate_kernel(const MergeDesc* __restrict__ md, const double* __restrict__ e,
                                                            double* ds, double* zsrt, const int64_t* __restrict__ perm,
                                                            int* typ, double* dk, double* zk, int64_t* kcol,
                                                            double* dval, int64_t* dcol, int64_t* rot_a, int64_t* rot_b,
                                                            double* rot_c, double* rot_s, int64_t* tpos,
                                                            MergeCounts* cnt) {
    __shared__ DeflLds s;
    const MergeDesc g = md[blockIdx.x];
    const int t = threadIdx.x;
    const int64_t o = g.o, N = g.N;
    const double rho2 = 2.0 * fabs(e[o + g.n1 - 1]);
    // tolerance: 8 eps max(max|d|, rho' max|z|)
    double mx = 0.0;
    for (int64_t i = t; i < N; i += DNT) mx = fmax(mx, fmax(fabs(ds[o + i]), rho2 * fabs(zsrt[o + i])));
    s.red[t] = mx;
    __syncthreads();
    for (int w = DNT / 2; w > 0; w >>= 1) {
        if (t < w) s.red[t] = fmax(s.red[t], s.red[t + w]);
        __syncthreads();
    }
    const double tol = 8.0 * EPS * s.red[0];
    // running totals (every thread) and the carried candidate (thread 0)
    int64_t K = 0, nd = 0, nr = 0;
    bool have = false;
    int64_t ccol = -1;
    double cd = 0.0, cz = 0.0;
    for (int64_t base = 0; base < N; base += DCH) {
        const int lim = (N - base) < DCH ? (int)(N - base) : DCH;
        __syncthreads();
        for (int q = t; q < lim; q += DNT) {
            s.sd[q] = ds[o + base + q];
            s.sz[q] = zsrt[o + base + q];
            s.sp[q] = perm[o + base + q];
        }
        __syncthreads();
        // (1) non-deflated poles of the chunk, in order
        int cntnd = 0;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int q = t * DPT + j;
            cntnd += (q < lim && rho2 * fabs(s.sz[q]) > tol) ? 1 : 0;
        }
        int64_t Mc64;
        int u = (int)defl_scan(cntnd, s, &Mc64);
        const int Mc = (int)Mc64;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int q = t * DPT + j;
            if (q < lim && rho2 * fabs(s.sz[q]) > tol) {
                s.L[u] = q;
                s.U[q] = u;
                ++u;
            }
        }
        __syncthreads();
        // (2) pairs (u-1, u) that rotate with original values
        int cntf = 0;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int v = t * DPT + j;
            if (v < Mc) {
                s.fate[v] = 0;
                s.hasrot[v] = 0;
            }
            if (v >= 1 && v < Mc) {
                double c, sn, r;
                const int qa = s.L[v - 1], qb = s.L[v];
                cntf += defl_rotates(s.sd[qa], s.sz[qa], s.sd[qb], s.sz[qb], tol, c, sn, r) ? 1 : 0;
            }
        }
        int64_t Fc64;
        int f = (int)defl_scan(cntf, s, &Fc64);
        const int Fc = (int)Fc64;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int v = t * DPT + j;
            if (v >= 1 && v < Mc) {
                double c, sn, r;
                const int qa = s.L[v - 1], qb = s.L[v];
                if (defl_rotates(s.sd[qa], s.sz[qa], s.sd[qb], s.sz[qb], tol, c, sn, r)) s.F[f++] = v;
            }
        }
        __syncthreads();
        // (3) the rotations and the chains after them (one thread)
        if (t == 0) s.keptc = 0;
        if (t == 0 && Mc > 0) {
            int settled = -1;      // every u <= settled has its test (u-1, u) decided
            bool endmod = false;   // a chain reached the chunk's last pole
            double endd = 0.0, endz = 0.0;
            // rotation deflating the pole before uu (column colp, state dp, zp)
            // into uu, then the tests that see uu's modified state
            auto rotate_from = [&](int uu, int64_t colp, double dp, double zp) {
                const int qb = s.L[uu];
                const double dj = s.sd[qb], zj = s.sz[qb];
                const int64_t col = s.sp[qb];
                double c, sn, r;
                defl_rotates(dp, zp, dj, zj, tol, c, sn, r);
                rot_a[o + nr] = colp;
                rot_b[o + nr] = col;
                rot_c[o + nr] = c;
                rot_s[o + nr] = sn;
                ++nr;
                if (typ[o + colp] != typ[o + col]) {
                    typ[o + colp] = 2;
                    typ[o + col] = 2;
                }
                s.hasrot[uu] = 1;
                s.rv[uu] = c * c * dp + sn * sn * dj;
                s.rcol[uu] = colp;
                double mdv = sn * sn * dp + c * c * dj, mzv = r;
                int v = uu + 1;
                for (; v < Mc; ++v) {
                    const int qv = s.L[v];
                    const double dv = s.sd[qv], zv = s.sz[qv];
                    const int64_t colv = s.sp[qv];
                    const int64_t colm = s.sp[s.L[v - 1]];
                    double c2, s2, r2;
                    if (!defl_rotates(mdv, mzv, dv, zv, tol, c2, s2, r2)) break;
                    rot_a[o + nr] = colm;
                    rot_b[o + nr] = colv;
                    rot_c[o + nr] = c2;
                    rot_s[o + nr] = s2;
                    ++nr;
                    if (typ[o + colm] != typ[o + colv]) {
                        typ[o + colm] = 2;
                        typ[o + colv] = 2;
                    }
                    s.fate[v - 1] = 2;
                    s.hasrot[v] = 1;
                    s.rv[v] = c2 * c2 * mdv + s2 * s2 * dv;
                    s.rcol[v] = colm;
                    mdv = s2 * s2 * mdv + c2 * c2 * dv;
                    mzv = r2;
                }
                if (v < Mc) {
                    // the test at v keeps pole v-1 with its modified state;
                    // pole v is original again
                    s.fate[v - 1] = 1;
                    s.kd[v - 1] = mdv;
                    s.kz[v - 1] = mzv;
                    settled = v;
                } else {
                    endmod = true;
                    endd = mdv;
                    endz = mzv;
                    settled = Mc - 1;
                }
            };
            // the candidate carried from the previous chunk against u = 0
            if (have) {
                const int q0 = s.L[0];
                double c, sn, r;
                if (defl_rotates(cd, cz, s.sd[q0], s.sz[q0], tol, c, sn, r)) {
                    rotate_from(0, ccol, cd, cz);
                } else {
                    dk[o + K] = cd;
                    zk[o + K] = cz;
                    kcol[o + K] = ccol;
                    s.keptc = 1;
                }
            }
            for (int fi = 0; fi < Fc; ++fi) {
                const int uu = s.F[fi];
                if (uu <= settled) continue;
                // pole uu-1 is original: no chain has reached it
                const int qa = s.L[uu - 1];
                s.fate[uu - 1] = 2;
                rotate_from(uu, s.sp[qa], s.sd[qa], s.sz[qa]);
            }
            // the chunk's last pole becomes the carried candidate
            const int ql = s.L[Mc - 1];
            ccol = s.sp[ql];
            cd = endmod ? endd : s.sd[ql];
            cz = endmod ? endz : s.sz[ql];
            have = true;
        }
        __syncthreads();
        K += s.keptc;
        // (4) kept poles u < Mc - 1 (the last one is carried)
        int cntk = 0;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int v = t * DPT + j;
            cntk += (v < Mc - 1 && s.fate[v] != 2) ? 1 : 0;
        }
        int64_t Kc;
        int64_t kpos = K + defl_scan(cntk, s, &Kc);
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int v = t * DPT + j;
            if (v < Mc - 1 && s.fate[v] != 2) {
                const int q = s.L[v];
                const bool m1 = s.fate[v] == 1;
                dk[o + kpos] = m1 ? s.kd[v] : s.sd[q];
                zk[o + kpos] = m1 ? s.kz[v] : s.sz[q];
                kcol[o + kpos] = s.sp[q];
                ++kpos;
            }
        }
        K += Kc;
        // deflated poles in scan order: a pole deflated by its own z, or the
        // candidate deflated by the rotation into this pole
        int cntd = 0;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int q = t * DPT + j;
            if (q < lim) cntd += (!(rho2 * fabs(s.sz[q]) > tol) || s.hasrot[s.U[q]]) ? 1 : 0;
        }
        int64_t Dc;
        int64_t dpos = nd + defl_scan(cntd, s, &Dc);
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int q = t * DPT + j;
            if (q >= lim) continue;
            if (!(rho2 * fabs(s.sz[q]) > tol)) {
                dval[o + dpos] = s.sd[q];
                dcol[o + dpos] = s.sp[q];
                ++dpos;
            } else if (s.hasrot[s.U[q]]) {
                const int v = s.U[q];
                dval[o + dpos] = s.rv[v];
                dcol[o + dpos] = s.rcol[v];
                ++dpos;
            }
        }
        nd += Dc;
        if (t == 0) s.sc[0] = nr;
        __syncthreads();
        nr = s.sc[0];
    }
    // the last candidate is kept
    if (t == 0 && have) {
        dk[o + K] = cd;
        zk[o + K] = cz;
        kcol[o + K] = ccol;
    }
    __syncthreads();
    if (t == 0) s.sc[0] = have ? 1 : 0;
    __syncthreads();
    K += s.sc[0];
    // the rotations' type changes and the kept columns are read back by
    // other threads: drain, barrier, drop stale vector-L1 lines
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    // kept columns by type (1 top only, 2 both, 3 bottom only) and each
    // one's position in type order: three counts packed in one prefix sum
    int64_t c1 = 0, c2 = 0, c3 = 0;
    {
        int64_t acc = 0;
        for (int64_t k0 = 0; k0 < K; k0 += DCH) {
            int64_t pk = 0;
#pragma unroll
            for (int j = 0; j < DPT; ++j) {
                const int64_t k = k0 + t * DPT + j;
                if (k < K) {
                    const int ty = typ[o + kcol[o + k]];
                    pk += (int64_t)1 << (21 * (ty - 1));
                }
            }
            int64_t tot;
            defl_scan(pk, s, &tot);
            acc += tot;
        }
        c1 = acc & 0x1FFFFF;
        c2 = (acc >> 21) & 0x1FFFFF;
        c3 = (acc >> 42) & 0x1FFFFF;
        int64_t run = 0;  // packed counts before the current chunk
        for (int64_t k0 = 0; k0 < K; k0 += DCH) {
            int64_t pk = 0;
            int tys[DPT];
#pragma unroll
            for (int j = 0; j < DPT; ++j) {
                const int64_t k = k0 + t * DPT + j;
                tys[j] = (k < K) ? typ[o + kcol[o + k]] : 0;
                if (k < K) pk += (int64_t)1 << (21 * (tys[j] - 1));
            }
            int64_t tot;
            int64_t before = run + defl_scan(pk, s, &tot);
#pragma unroll
            for (int j = 0; j < DPT; ++j) {
                const int64_t k = k0 + t * DPT + j;
                if (k < K) {
                    const int ty = tys[j];
                    const int64_t p1 = before & 0x1FFFFF, p2 = (before >> 21) & 0x1FFFFF,
                                  p3 = (before >> 42) & 0x1FFFFF;
                    tpos[o + k] = (ty == 1) ? p1 : (ty == 2) ? c1 + p2 : c1 + c2 + p3;
                    before += (int64_t)1 << (21 * (ty - 1));
                }
            }
            run += tot;
        }
    }
    if (t == 0) {
        MergeCounts mc;
        mc.K = K;
        mc.ndefl = nd;
        mc.nrot = nr;
        mc.c1 = c1;
        mc.c2 = c2;
        mc.c3 = c3;
        mc.rho2 = rho2;
        cnt[blockIdx.x] = mc;
    }
}

// apply the deflation rotations to the columns of the merged block (one row per thread)
__global__ __launch_bounds__(256) void merge_rotate_kernel(const MergeDesc* __restrict__ md, const MergeCounts* __restrict__ cnt,
                                                           const int64_t* __restrict__ rot_a, const int64_t* __restrict__ rot_b,
                                                           const double* __restrict__ rot_c, const double* __restrict__ rot_s,
                                                           double* Z, int64_t ldz) {
    const MergeDesc g = md[blockIdx.y];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= g.N) return;
    const int64_t nr = cnt[blockIdx.y].nrot;
    double* zr = Z + g.o + r;
    for (int64_t q = 0; q < nr; ++q) {
        int64_t a = g.o + rot_a[g.o + q], b = g.o + rot_b[g.o + q];
        double c = rot_c[g.o + q], s = rot_s[g.o + q];
        double x = zr[a * ldz], y = zr[b * ldz];
        zr[a * ldz] = c * x - s * y;
        zr[b * ldz] = s * x + c * y;
    }
}

// Secular equation: one thread per root.  Root k is stored as its nearer
// pole org_k and the offset tau_k, so that d_j - lambda_k = (d_j - d_org) - tau
// is available to full relative accuracy wherever it is needed.  The poles
// and rho z_j^2 are streamed through LDS in tiles shared by the workgroup;
// each thread sums in ascending j as a plain loop would, and the workgroup
// iterates until all its roots have converged.
constexpr int STILE = 1024;
constexpr int SNT = 256;
constexpr int SRL = 8;             // lanes per root: each sums every eighth pole
constexpr int SRW = SNT / SRL;     // roots per workgroup
__global__ __launch_bounds__(SNT) void merge_secular_kernel(const MergeDesc* __restrict__ md, const MergeCounts* __restrict__ cnt,
                                                            const double* __restrict__ dk, const double* __restrict__ zk,
                                                            int64_t* rorg, double* rtau, double* lam, int* fail) {
    __shared__ double sd[STILE], sw[STILE], sz[STILE];  // d_j, (rho z_j) z_j, z_j
    const MergeDesc g = md[blockIdx.y];
    const int64_t K = cnt[blockIdx.y].K;
    if ((int64_t)blockIdx.x * SRW >= K) return;  // uniform over the workgroup
    // SRL adjacent lanes share root k and split its sums over the poles (the
    // partial sums are combined by lane exchanges, so all of them hold the
    // same totals and take the same steps)
    const int sub = threadIdx.x & (SRL - 1);
    const int64_t k = (int64_t)blockIdx.x * SRW + (threadIdx.x / SRL);
    const bool act = k < K;
    const double rho = cnt[blockIdx.y].rho2;
    const double* d = dk + g.o;
    const double* z = zk + g.o;
    // sum over j of fn(j, d_j, w_j) in ascending j, tile by tile (every thread of the workgroup calls this)
    auto stream = [&](auto&& fn) {
        for (int64_t base = 0; base < K; base += STILE) {
            __syncthreads();
            for (int q = threadIdx.x; q < STILE; q += SNT) {
                const int64_t j = base + q;
                if (j < K) {
                    sd[q] = d[j];
                    sw[q] = rho * z[j] * z[j];
                    sz[q] = z[j];
                }
            }
            __syncthreads();
            const int lim = (int)((K - base) < STILE ? (K - base) : STILE);
            fn(base, lim);
        }
    };
    const int64_t kk = act ? k : 0;
    // bracket: the sign of f at the midpoint between d_k and d_k+1 picks the
    // nearer pole; the last root lies in (d_K-1, d_K-1 + rho |z|^2).  Both
    // sums run in the same (workgroup-uniform) pass over the tiles.
    const bool last = kk >= K - 1;
    const double dkk = d[kk];
    const double mid = last ? 0.0 : 0.5 * (d[kk + 1] - dkk);
    double f0 = 0.0, zz = 0.0;
    stream([&](int64_t, int lim) {
        if (!last)
            for (int q = sub; q < lim; q += SRL) f0 += sw[q] / ((sd[q] - dkk) - mid);
        else
            for (int q = sub; q < lim; q += SRL) zz += sz[q] * sz[q];
    });
#pragma unroll
    for (int o = 1; o < SRL; o <<= 1) {
        f0 += __shfl_xor(f0, o, 64);
        zz += __shfl_xor(zz, o, 64);
    }
    f0 += 1.0;
    int64_t org;
    double lo, hi;
    if (!last) {
        if (f0 >= 0.0) {
            org = kk;
            lo = 0.0;
            hi = mid;
        } else {
            org = kk + 1;
            lo = -mid;
            hi = 0.0;
        }
    } else {
        org = kk;
        lo = 0.0;
        hi = rho * zz;
    }
    const double dorg = d[org];
    const double Dk = d[kk] - dorg;
    const double Dk1 = (kk < K - 1) ? d[kk + 1] - dorg : 0.0;
    double x = 0.5 * (lo + hi);
    bool done = !act;
    bool converged = false;
    for (int it = 0; it < 400; ++it) {
        if (!__syncthreads_or(done ? 0 : 1)) break;
        double psi = 0.0, phi = 0.0, dpsi = 0.0, dphi = 0.0;
        stream([&](int64_t base, int lim) {
            if (done) return;
            // j <= kk contributes to psi, j > kk to phi
            const int split = (int)std::min<int64_t>(std::max<int64_t>(kk + 1 - base, 0), lim);
            // one division per pole: t = w / dl and t / dl from 1 / dl
            // (two roundings each, well inside the stopping test's 8 eps)
            for (int q = sub; q < lim; q += SRL) {
                const double rl = 1.0 / ((sd[q] - dorg) - x);
                const double tq = sw[q] * rl;
                if (q < split) {
                    psi += tq;
                    dpsi += tq * rl;
                } else {
                    phi += tq;
                    dphi += tq * rl;
                }
            }
        });
#pragma unroll
        for (int o = 1; o < SRL; o <<= 1) {
            psi += __shfl_xor(psi, o, 64);
            phi += __shfl_xor(phi, o, 64);
            dpsi += __shfl_xor(dpsi, o, 64);
            dphi += __shfl_xor(dphi, o, 64);
        }
        if (done) continue;
        const double f = 1.0 + psi + phi;
        if (f < 0.0)
            lo = x;
        else
            hi = x;
        if (fabs(f) <= 8.0 * EPS * (1.0 + fabs(psi) + fabs(phi)) ||
            hi - lo <= 2.0 * EPS * fmax(fabs(lo), fabs(hi))) {
            converged = true;
            done = true;
            continue;
        }
        // two-pole rational model through f, f' (poles d_k, d_k+1), safeguarded by the bracket
        const double dlk = Dk - x;
        const double bb = dpsi * dlk * dlk;
        double a2, a1, a0;
        if (kk < K - 1) {
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
    if (!act || sub != 0) return;
    if (!converged) *fail = 2;
    lam[g.o + k] = dorg + x;
    rorg[g.o + k] = org;
    rtau[g.o + k] = x;
}

// zhat_j from the roots (products paired so that every factor lies in (0, 1]).
__global__ __launch_bounds__(256) void merge_zhat_kernel(const MergeDesc* __restrict__ md, const MergeCounts* __restrict__ cnt,
                                                         const double* __restrict__ dk, const double* __restrict__ zk,
                                                         const int64_t* __restrict__ rorg, const double* __restrict__ rtau,
                                                         double* zh) {
    const MergeDesc g = md[blockIdx.y];
    const int64_t K = cnt[blockIdx.y].K;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K) return;
    const double rho = cnt[blockIdx.y].rho2;
    const double* d = dk + g.o;
    const int64_t* org = rorg + g.o;
    const double* tau = rtau + g.o;
    const double dj = d[j];
    // lambda_k - d_j = tau_k - (d_j - d_org(k))
    double p = (tau[K - 1] - (dj - d[org[K - 1]])) / rho;
    for (int64_t k = 0; k < j; ++k) p *= (tau[k] - (dj - d[org[k]])) / (d[k] - dj);
    for (int64_t k = j; k < K - 1; ++k) p *= (tau[k] - (dj - d[org[k]])) / (d[k + 1] - dj);
    zh[g.o + j] = copysign(sqrt(fabs(p)), zk[g.o + j]);
}

// column k of U: zhat / (d - lambda_k), normalised (stored K x K, ld K)
__global__ __launch_bounds__(256) void merge_vec_kernel(const MergeDesc* __restrict__ md, const MergeCounts* __restrict__ cnt,
                                                        int64_t Nmax, const double* __restrict__ dk,
                                                        const int64_t* __restrict__ rorg, const double* __restrict__ rtau,
                                                        const double* __restrict__ zh, double* DU) {
    __shared__ double red[256];
    const MergeDesc g = md[blockIdx.y];
    const int64_t K = cnt[blockIdx.y].K;
    const int64_t k = blockIdx.x;
    if (k >= K) return;
    double* col = DU + g.o * Nmax + k * K;
    const double* d = dk + g.o;
    const double dorg = d[rorg[g.o + k]], tau = rtau[g.o + k];
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < K; j += 256) {
        double u = zh[g.o + j] / ((d[j] - dorg) - tau);
        col[j] = u;
        s += u * u;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double inv = 1.0 / sqrt(red[0]);
    for (int64_t j = threadIdx.x; j < K; j += 256) col[j] *= inv;
}

// Gather the kept columns of Q in type order (Qsel), U's rows in the same
// order (Ut), and the deflated columns into Znew[:, K..N).
__global__ __launch_bounds__(256) void merge_gather_kernel(const MergeDesc* __restrict__ md, const MergeCounts* __restrict__ cnt,
                                                           const double* __restrict__ Z, int64_t ldz,
                                                           const int64_t* __restrict__ kcol, const int64_t* __restrict__ tpos,
                                                           const int64_t* __restrict__ dcol, int64_t Nmax,
                                                           const double* __restrict__ DU, double* Ut, double* Qsel,
                                                           double* Znew) {
    const MergeDesc g = md[blockIdx.z];
    const MergeCounts c = cnt[blockIdx.z];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t col = blockIdx.y; col < g.N; col += gridDim.y) {
        if (col < c.K) {
            if (r < g.N) {
                int64_t src = g.o + kcol[g.o + col];
                Qsel[g.o * Nmax + r + tpos[g.o + col] * g.N] = Z[(g.o + r) + src * ldz];
            }
            // Ut row tpos[j] = U row j, for column `col` of U
            if (r < c.K) Ut[g.o * Nmax + tpos[g.o + r] + col * c.K] = DU[g.o * Nmax + r + col * c.K];
        } else {
            if (r < g.N) {
                int64_t src = g.o + dcol[g.o + (col - c.K)];
                Znew[g.o * Nmax + r + col * g.N] = Z[(g.o + r) + src * ldz];
            }
        }
    }
}

__global__ void merge_gemm_setup_kernel(int nm, const MergeDesc* __restrict__ md, const MergeCounts* __restrict__ cnt,
                                        int64_t Nmax, double* Ut, double* Qsel, double* Znew, GemmProblem* pr) {
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nm) return;
    const MergeDesc g = md[m];
    const MergeCounts c = cnt[m];
    double* q = Qsel + g.o * Nmax;
    double* u = Ut + g.o * Nmax;
    double* zn = Znew + g.o * Nmax;
    // top rows: Q[0:n1, type 1|2] Ut[type 1|2, :]
    pr[2 * m] = GemmProblem{g.n1, c.K, c.c1 + c.c2, q, g.N, u, c.K > 0 ? c.K : 1, zn, g.N, 1.0, 0.0};
    // bottom rows: Q[n1:N, type 2|3] Ut[type 2|3, :]
    pr[2 * m + 1] = GemmProblem{g.N - g.n1, c.K, c.c2 + c.c3, q + g.n1 + c.c1 * g.N, g.N, u + c.c1,
                                c.K > 0 ? c.K : 1, zn + g.n1, g.N, 1.0, 0.0};
}

// output values of a merge: the roots, then the deflated poles (ranked by the next kernel)
__global__ __launch_bounds__(256) void merge_values_kernel(const MergeDesc* __restrict__ md, const MergeCounts* __restrict__ cnt,
                                                           const double* __restrict__ lam, const double* __restrict__ dval,
                                                           double* vals) {
    const MergeDesc g = md[blockIdx.y];
    const int64_t K = cnt[blockIdx.y].K;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((int64_t)blockIdx.x * blockDim.x >= g.N) return;
    // assemble the value list in vals[o .. o+N)
    if (i < g.N) vals[g.o + i] = (i < K) ? lam[g.o + i] : dval[g.o + (i - K)];
}

__global__ __launch_bounds__(256) void merge_rank2_kernel(const MergeDesc* __restrict__ md, const double* __restrict__ vals,
                                                          int64_t* rank) {
    __shared__ double tile[1024];
    const MergeDesc g = md[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((int64_t)blockIdx.x * blockDim.x >= g.N) return;
    double vi = (i < g.N) ? vals[g.o + i] : 0.0;
    int64_t r = rank_of(vals + g.o, g.N, i, vi, tile);
    if (i < g.N) rank[g.o + i] = r;
}

__global__ __launch_bounds__(256) void merge_scatter_kernel(const MergeDesc* __restrict__ md, int64_t Nmax,
                                                            const double* __restrict__ vals, const int64_t* __restrict__ rank,
                                                            const double* __restrict__ Znew, double* D, double* Z,
                                                            int64_t ldz) {
    const MergeDesc g = md[blockIdx.z];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t col = blockIdx.y; col < g.N; col += gridDim.y) {
        int64_t dst = g.o + rank[g.o + col];
        if (r < g.N) Z[(g.o + r) + dst * ldz] = Znew[g.o * Nmax + r + col * g.N];
        if (r == 0) D[dst] = vals[g.o + col];
    }
}

// final ascending sort of the whole spectrum is already the root's order; a
// single leaf needs its own sort
__global__ __launch_bounds__(256) void sort_single_kernel(int64_t n, const double* __restrict__ D, int64_t* rank) {
    __shared__ double tile[1024];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double vi = (i < n) ? D[i] : 0.0;
    int64_t r = rank_of(D, n, i, vi, tile);
    if (i < n) rank[i] = r;
}

__global__ __launch_bounds__(256) void permute_cols_kernel(int64_t n, const int64_t* __restrict__ rank,
                                                           const double* __restrict__ Din, const double* __restrict__ Zin,
                                                           int64_t ldin, double* Dout, double* Zout, int64_t ldout) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t col = blockIdx.y; col < n; col += gridDim.y) {
        int64_t dst = rank[col];
        if (r < n) Zout[r + dst * ldout] = Zin[r + col * ldin];
        if (r == 0) Dout[dst] = Din[col];
    }
}

struct Tree {
    std::vector<int64_t> leaf_lo;
    std::vector<int> leaf_m;
    std::vector<int64_t> splits;
    std::vector<std::vector<MergeDesc>> levels;  // deepest first
};

void build_tree(int64_t lo, int64_t hi, int leaf, int depth, Tree& T, std::vector<std::vector<MergeDesc>>& bydepth) {
    int64_t N = hi - lo;
    if (N <= leaf) {
        T.leaf_lo.push_back(lo);
        T.leaf_m.push_back((int)N);
        return;
    }
    int64_t n1 = N / 2;
    T.splits.push_back(lo + n1 - 1);
    if ((int)bydepth.size() <= depth) bydepth.resize(depth + 1);
    bydepth[depth].push_back(MergeDesc{lo, N, n1});
    build_tree(lo, lo + n1, leaf, depth + 1, T, bydepth);
    build_tree(lo + n1, hi, leaf, depth + 1, T, bydepth);
}

inline unsigned gy(int64_t v) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(v, 65535)); }

}  // namespace

// Divide and conquer on (d, e): d := eigenvalues ascending, Z := eigenvectors.
// Synchronous (allocates its workspace).  Returns FL_OK / FL_ENOCONV / FL_EHIP / FL_ENOMEM.
int fl_stedc_device(fl_ctx* ctx, int64_t n, double* d, const double* e, double* Zout, int64_t ldz, int leaf) {
    hipStream_t s = ctx->stream;
    if (n <= 0) return FL_OK;
    if (leaf <= 1 || leaf > LEAF_MAX) leaf = 32;
    Tree T;
    std::vector<std::vector<MergeDesc>> bydepth;
    build_tree(0, n, leaf, 0, T, bydepth);
    int64_t nlev = (int64_t)bydepth.size();
    int64_t Nmax_all = n;
    // workspace
    DevBuf bZ, bDU, bUt, bQ, bZn, bvec, bint, bleaf, bmd, bcnt, bpr, bfail, bsplit;
    size_t nn = (size_t)n * (size_t)Nmax_all;
    const int64_t ldw = n;  // Z work array is n x n
    FL_HIP(ctx, bZ.alloc(sizeof(double) * (size_t)n * n));
    double* Z = bZ.as<double>();
    if (nlev > 0) {
        FL_HIP(ctx, bDU.alloc(sizeof(double) * nn));
        FL_HIP(ctx, bUt.alloc(sizeof(double) * nn));
        FL_HIP(ctx, bQ.alloc(sizeof(double) * nn));
        FL_HIP(ctx, bZn.alloc(sizeof(double) * nn));
    }
    // double arrays: ds zsrt dk zk dval rot_c rot_s lam zh vals rtau (11 n)
    FL_HIP(ctx, bvec.alloc(sizeof(double) * 11 * (size_t)n));
    double* ds = bvec.as<double>();
    double* zsrt = ds + n;
    double* dk = zsrt + n;
    double* zk = dk + n;
    double* dval = zk + n;
    double* rc = dval + n;
    double* rs = rc + n;
    double* lam = rs + n;
    double* zh = lam + n;
    double* vals = zh + n;
    double* rtau = vals + n;
    // int64 arrays: perm kcol dcol rot_a rot_b tpos rank rorg (8 n) + typ (int)
    FL_HIP(ctx, bint.alloc(sizeof(int64_t) * 8 * (size_t)n + sizeof(int) * (size_t)n));
    int64_t* perm = bint.as<int64_t>();
    int64_t* kcol = perm + n;
    int64_t* dcol = kcol + n;
    int64_t* ra = dcol + n;
    int64_t* rb = ra + n;
    int64_t* tpos = rb + n;
    int64_t* rank = tpos + n;
    int64_t* rorg = rank + n;
    int* typ = (int*)(rorg + n);
    FL_HIP(ctx, bfail.alloc(sizeof(int)));
    int* fail = bfail.as<int>();
    FL_HIP(ctx, hipMemsetAsync(fail, 0, sizeof(int), s));

    // leaves
    size_t nleaf = T.leaf_lo.size();
    FL_HIP(ctx, bleaf.alloc((sizeof(int64_t) + sizeof(int)) * nleaf));
    int64_t* dleaf_lo = bleaf.as<int64_t>();
    int* dleaf_m = (int*)(dleaf_lo + nleaf);
    FL_HIP(ctx, hipMemcpyAsync(dleaf_lo, T.leaf_lo.data(), sizeof(int64_t) * nleaf, hipMemcpyHostToDevice, s));
    FL_HIP(ctx, hipMemcpyAsync(dleaf_m, T.leaf_m.data(), sizeof(int) * nleaf, hipMemcpyHostToDevice, s));
    FL_HIP(ctx, hipMemsetAsync(Z, 0, sizeof(double) * (size_t)n * n, s));
    if (!T.splits.empty()) {
        FL_HIP(ctx, bsplit.alloc(sizeof(int64_t) * T.splits.size()));
        FL_HIP(ctx, hipMemcpyAsync(bsplit.p, T.splits.data(), sizeof(int64_t) * T.splits.size(), hipMemcpyHostToDevice, s));
        split_adjust_kernel<<<1, 1, 0, s>>>(bsplit.as<int64_t>(), (int)T.splits.size(), d, e);
        FL_HIP(ctx, hipGetLastError());
    }
    leaf_kernel<<<(unsigned)nleaf, 64, 0, s>>>(dleaf_lo, dleaf_m, d, e, Z, ldw, fail);
    FL_HIP(ctx, hipGetLastError());

    // merges, deepest level first
    size_t maxm = 0;
    for (auto& L : bydepth) maxm = std::max(maxm, L.size());
    if (nlev > 0) {
        FL_HIP(ctx, bmd.alloc(sizeof(MergeDesc) * maxm * nlev));
        FL_HIP(ctx, bcnt.alloc(sizeof(MergeCounts) * maxm));
        FL_HIP(ctx, bpr.alloc(sizeof(GemmProblem) * 2 * maxm));
    }
    MergeCounts* cnt = bcnt.as<MergeCounts>();
    GemmProblem* pr = bpr.as<GemmProblem>();
    for (int64_t lev = nlev - 1; lev >= 0; --lev) {
        const auto& L = bydepth[lev];
        int nm = (int)L.size();
        MergeDesc* md = bmd.as<MergeDesc>() + lev * maxm;
        FL_HIP(ctx, hipMemcpyAsync(md, L.data(), sizeof(MergeDesc) * nm, hipMemcpyHostToDevice, s));
        int64_t Nmax = 0;
        for (auto& g : L) Nmax = std::max(Nmax, g.N);
        const unsigned bx = (unsigned)FL_DIV_UP(Nmax, 256);
        merge_sort_kernel<<<dim3(bx, nm), 256, 0, s>>>(md, d, Z, ldw, e, ds, zsrt, perm, typ);
        FL_HIP(ctx, hipGetLastError());
        merge_deflate_kernel<<<nm, DNT, 0, s>>>(md, e, ds, zsrt, perm, typ, dk, zk, kcol, dval, dcol, ra, rb, rc, rs,
                                                tpos, cnt);
        FL_HIP(ctx, hipGetLastError());
        merge_rotate_kernel<<<dim3(bx, nm), 256, 0, s>>>(md, cnt, ra, rb, rc, rs, Z, ldw);
        FL_HIP(ctx, hipGetLastError());
        merge_secular_kernel<<<dim3((unsigned)FL_DIV_UP(Nmax, SRW), nm), SNT, 0, s>>>(md, cnt, dk, zk, rorg, rtau,
                                                                                      lam, fail);
        FL_HIP(ctx, hipGetLastError());
        merge_zhat_kernel<<<dim3(bx, nm), 256, 0, s>>>(md, cnt, dk, zk, rorg, rtau, zh);
        FL_HIP(ctx, hipGetLastError());
        merge_vec_kernel<<<dim3((unsigned)Nmax, nm), 256, 0, s>>>(md, cnt, Nmax, dk, rorg, rtau, zh, bDU.as<double>());
        FL_HIP(ctx, hipGetLastError());
        merge_gather_kernel<<<dim3(bx, gy(Nmax), nm), 256, 0, s>>>(md, cnt, Z, ldw, kcol, tpos, dcol, Nmax,
                                                                   bDU.as<double>(), bUt.as<double>(), bQ.as<double>(),
                                                                   bZn.as<double>());
        FL_HIP(ctx, hipGetLastError());
        merge_gemm_setup_kernel<<<FL_DIV_UP(nm, 64), 64, 0, s>>>(nm, md, cnt, Nmax, bUt.as<double>(), bQ.as<double>(),
                                                                  bZn.as<double>(), pr);
        FL_HIP(ctx, hipGetLastError());
        FL_HIP(ctx, fl_dgemm_batched(s, 0, 0, pr, 2 * nm, Nmax, Nmax));
        merge_values_kernel<<<dim3(bx, nm), 256, 0, s>>>(md, cnt, lam, dval, vals);
        FL_HIP(ctx, hipGetLastError());
        merge_rank2_kernel<<<dim3(bx, nm), 256, 0, s>>>(md, vals, rank);
        FL_HIP(ctx, hipGetLastError());
        merge_scatter_kernel<<<dim3(bx, gy(Nmax), nm), 256, 0, s>>>(md, Nmax, vals, rank, bZn.as<double>(), d, Z, ldw);
        FL_HIP(ctx, hipGetLastError());
    }
    // Z -> Zout (sorted ascending; the root merge already produced ascending
    // order, a lone leaf needs its own sort)
    {
        const unsigned bx = (unsigned)FL_DIV_UP(n, 256);
        sort_single_kernel<<<bx, 256, 0, s>>>(n, d, rank);
        FL_HIP(ctx, hipGetLastError());
        permute_cols_kernel<<<dim3(bx, gy(n)), 256, 0, s>>>(n, rank, d, Z, ldw, ds, Zout, ldz);
        FL_HIP(ctx, hipGetLastError());
        FL_HIP(ctx, hipMemcpyAsync(d, ds, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
    int hfail = 0;
    FL_HIP(ctx, hipMemcpyAsync(&hfail, fail, sizeof(int), hipMemcpyDeviceToHost, s));
    FL_HIP(ctx, hipStreamSynchronize(s));
    if (hfail) return fl_fail(ctx, FL_ENOCONV, hfail == 1 ? "stedc: QL leaf did not converge" : "stedc: secular equation did not converge");
    return FL_OK;
}
