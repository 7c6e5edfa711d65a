// All eigenpairs in an interval by spectrum slicing (Sections "Solving for
// all eigenpairs in an interval", "Partitioning" with its greedy
// partitioning, and "Post-processing"), for pencils held only in sparse
// form.
//
//  1. Counting: nu(sigma) = number of eigenvalues below sigma from the
//     inertia of K - sigma M (fl_inertia_count); the interval holds
//     nu(hi) - nu(lo) eigenvalues.
//  2. Greedy partitioning: split points start evenly spaced; each round
//     counts below every split point at once (one launch, one workgroup per
//     shift) and moves the points so that the piecewise-linear cumulative
//     count through the measured points would give equal loads; the best
//     partition over n_a rounds is kept, and a slice still above the load
//     limit is halved (counted again) until none is.
//  3. Every slice is an independent "evaluator": its shifted pencil
//     K - sigma_s M (sigma_s = slice midpoint) is factored once (banded
//     LDL^T, kept in two layouts), and shift-invert subspace iteration with
//     a block of p_s = 2 m_s + 16 vectors runs for all slices together:
//       Y_s = (K - sigma_s M)^-1 M X_s   (banded solves, 8 columns per
//       64-lane block, and one step of iterative refinement: the pivots of
//       an LDL^T without pivoting of an indefinite matrix can grow, and the
//       refinement keeps the solves backward stable, Skeel 1980, so that
//       the subspace converges to the pencil's eigenvectors, not to those of
//       the factorisation's perturbed pencil);  columns of Y scaled to unit
//       M-norm;  Rayleigh-Ritz
//       of (Y^T K Y, Y^T M Y) per slice by the batched eigensolver;
//       X_s = Y_s Z_s.
//     A slice has converged when exactly m_s of its Ritz pairs lie in it
//     with residuals ||K x - theta M x|| below tol theta ||M x|| (the m_s
//     eigenvalues inside are known from the counts; Ritz values of the
//     unconverged guard directions are mixtures and may fall anywhere).
//  4. Post-processing: the converged Ritz pairs inside each slice are the
//     slice's eigenpairs, M-orthonormal within the slice (Rayleigh-Ritz with
//     an M-orthonormal Z); equal eigenvalues never straddle a split point
//     (each split is a count boundary), and eigenvectors of different slices
//     belong to different eigenvalues, orthogonal up to residual / gap; one
//     Newton-Schulz step V := V (3 I - V^T M V) / 2 over all of them removes
//     that to second order.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>
#include "internal.h"

namespace {

constexpr int SOLVE_COLS = 8;   // right-hand sides per 64-lane block
constexpr int SUB = 8;          // lanes per right-hand side
constexpr int RING = 512;       // > FL_BAND_MAX: the last bw solution entries of each column

struct SliceSolve {
    const double* Lcol;  // column layout: L(r, c) at (r - c) + c ldb, D on the diagonal
    const double* Lrow;  // row layout: L(r, c) at (bw - (r - c)) + r ldb
    double* X;           // n x ncols block (column-major, ld n), solved in place
    int ncols;
};

// (L D L^T) X = X for every slice's block: one 64-lane block per 8 columns
// (lane = 8 column + sub), the 8 lanes of a column split each row's sum.
// Forward L y = b by rows (row layout), z = D^-1 y, backward L^T x = z by
// rows (column layout); each column's last bw values sit in an LDS ring.
__global__ __launch_bounds__(64) void band_solve_kernel(int64_t n, int bw, int64_t ldb, const SliceSolve* sl,
                                                        const int* blk_slice, const int* blk_col) {
    __shared__ double ring[SOLVE_COLS][RING];
    const int lane = threadIdx.x, c = lane / SUB, sub = lane % SUB;
    const SliceSolve S = sl[blk_slice[blockIdx.x]];
    const int col = blk_col[blockIdx.x] + c;
    const bool live = col < S.ncols;
    double* x = S.X + (int64_t)(live ? col : S.ncols - 1) * n;
    // forward: y_i = b_i - sum_{j in [i - bw, i)} L(i, j) y_j;  x_i := y_i / D_i
    for (int64_t i = 0; i < n; ++i) {
        const int64_t jlo = i - bw > 0 ? i - bw : 0;
        const double* lr = S.Lrow + i * ldb + bw - i;  // lr[j] = L(i, j)
        double part = 0.0;
        for (int64_t j = jlo + sub; j < i; j += SUB) part += lr[j] * ring[c][j & (RING - 1)];
        part += __shfl_xor(part, 4, 64);
        part += __shfl_xor(part, 2, 64);
        part += __shfl_xor(part, 1, 64);
        if (sub == 0) {
            const double y = x[i] - part;
            ring[c][i & (RING - 1)] = y;
            if (live) x[i] = y / lr[i];
        }
        __syncthreads();
    }
    __syncthreads();
    // backward: x_i = z_i - sum_{j in (i, i + bw]} L(j, i) x_j
    for (int64_t i = n - 1; i >= 0; --i) {
        const int64_t jhi = i + bw < n - 1 ? i + bw : n - 1;
        const double* lc = S.Lcol + i * ldb - i;  // lc[j] = L(j, i)
        double part = 0.0;
        for (int64_t j = i + 1 + sub; j <= jhi; j += SUB) part += lc[j] * ring[c][j & (RING - 1)];
        part += __shfl_xor(part, 4, 64);
        part += __shfl_xor(part, 2, 64);
        part += __shfl_xor(part, 1, 64);
        if (sub == 0) {
            const double v = x[i] - part;
            ring[c][i & (RING - 1)] = v;
            if (live) x[i] = v;
        }
        __syncthreads();
    }
}

// Gather / scatter between the natural and the banded numbering:
// Xp[pinv[i] + k n] = X[i + k n] (TO_BAND), X[i + k n] = Xp[pinv[i] + k n]
// (FROM_BAND) or X[i + k n] += Xp[pinv[i] + k n] (ADD_FROM_BAND).
enum { TO_BAND = 0, FROM_BAND = 1, ADD_FROM_BAND = 2 };
__global__ void permute_rows_kernel(int64_t n, int64_t ncols, const int32_t* __restrict__ pinv,
                                    const double* __restrict__ src, double* __restrict__ dst, int mode) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t pi = pinv[i];
    for (int64_t k = blockIdx.y; k < ncols; k += gridDim.y) {
        if (mode == TO_BAND)
            dst[pi + k * n] = src[i + k * n];
        else if (mode == FROM_BAND)
            dst[i + k * n] = src[pi + k * n];
        else
            dst[i + k * n] += src[pi + k * n];
    }
}

// R = B - (K - sigma_c M) Y for CSR K and M on one pattern, sigma_c the
// shift of column c's slice: the residual of the banded solves, for one step
// of iterative refinement.  A thread takes one row and 8 columns.
constexpr int RES_COLS = 8;
__global__ void shifted_residual_kernel(int64_t n, const int32_t* __restrict__ rowptr,
                                        const int32_t* __restrict__ colidx, const double* __restrict__ kval,
                                        const double* __restrict__ mval, int64_t ncols,
                                        const double* __restrict__ sigma, const double* __restrict__ B,
                                        const double* __restrict__ Y, double* __restrict__ R) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t p0 = rowptr[i], p1 = rowptr[i + 1];
    for (int64_t c0 = (int64_t)blockIdx.y * RES_COLS; c0 < ncols; c0 += (int64_t)gridDim.y * RES_COLS) {
        const int nc = (int)((ncols - c0) < RES_COLS ? (ncols - c0) : RES_COLS);
        double sk[RES_COLS], sm[RES_COLS];
#pragma unroll
        for (int c = 0; c < RES_COLS; ++c) sk[c] = sm[c] = 0.0;
        for (int32_t p = p0; p < p1; ++p) {
            const double kv = kval[p], mv = mval[p];
            const double* y = Y + colidx[p] + c0 * n;
#pragma unroll
            for (int c = 0; c < RES_COLS; ++c)
                if (c < nc) {
                    sk[c] += kv * y[c * n];
                    sm[c] += mv * y[c * n];
                }
        }
#pragma unroll
        for (int c = 0; c < RES_COLS; ++c)
            if (c < nc) R[i + (c0 + c) * n] = B[i + (c0 + c) * n] - (sk[c] - sigma[c0 + c] * sm[c]);
    }
}

// Start block: entries from SplitMix64 (Steele, Lea and Flood) of the global
// index, mapped to (-1, 1).
__global__ void start_block_kernel(int64_t count, uint64_t seed, double* X) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        X[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
}

// Relative residual of every Ritz pair: ||KX_j - theta_j MX_j|| /
// (max(|theta_j|, scale_j) ||MX_j||), scale_j = the upper end of the column's
// slice (for the lowest modes of a slice the rounding of K x is of the size
// of the slice's largest eigenvalues), one block per column (fixed-order
// reduction).
__global__ __launch_bounds__(256) void ritz_residual_kernel(int64_t n, const double* __restrict__ KX,
                                                            const double* __restrict__ MX,
                                                            const double* __restrict__ theta,
                                                            const double* __restrict__ scale, double* rel) {
    __shared__ double ra[256], rb[256];
    const int64_t j = blockIdx.x;
    const double th = theta[j];
    double sa = 0.0, sb = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double m = MX[i + j * n];
        const double r = KX[i + j * n] - th * m;
        sa += r * r;
        sb += m * m;
    }
    ra[threadIdx.x] = sa;
    rb[threadIdx.x] = sb;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            ra[threadIdx.x] += ra[threadIdx.x + w];
            rb[threadIdx.x] += rb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) rel[j] = sqrt(ra[0]) / (fmax(fabs(th), scale[j]) * sqrt(rb[0]) + 1e-300);
}

// y_j := y_j / sqrt(y_j^T (M y)_j) for the columns of Y, and the same scale
// on K Y and M Y (one block per column): the projected pencils are formed
// from M-normalised columns, whose lengths after a shift-invert step differ
// by the spread of 1 / |theta - sigma|.
__global__ __launch_bounds__(256) void mnormalise_kernel(int64_t n, double* Y, double* KY, double* MY) {
    __shared__ double red[256];
    const int64_t j = blockIdx.x;
    double sacc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) sacc += Y[i + j * n] * MY[i + j * n];
    red[threadIdx.x] = sacc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double f = red[0] > 0.0 ? 1.0 / sqrt(red[0]) : 1.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        Y[i + j * n] *= f;
        KY[i + j * n] *= f;
        MY[i + j * n] *= f;
    }
}

// out column q = X column idx[q], theta_out[q] = theta[idx[q]].
__global__ void gather_pairs_kernel(int64_t n, int64_t m, const int64_t* __restrict__ idx,
                                    const double* __restrict__ X, const double* __restrict__ th, double* V,
                                    int64_t ldv, double* theta) {
    for (int64_t q = blockIdx.y; q < m; q += gridDim.y) {
        const int64_t src = idx[q];
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
            V[i + q * ldv] = X[i + src * n];
        if (blockIdx.x == 0 && threadIdx.x == 0) theta[q] = th[src];
    }
}

// H = (3 I - G) / 2 for the m x m Gram matrix G (in place): one
// Newton-Schulz step towards M-orthonormal columns, V := V H.
__global__ void newton_schulz_kernel(int64_t m, double* G) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    for (int64_t j = blockIdx.y; j < m; j += gridDim.y) G[i + j * m] = (i == j ? 1.5 : 0.0) - 0.5 * G[i + j * m];
}

struct Slice {
    double a, b;     // [a, b)
    int64_t m;       // eigenvalues inside
    int64_t p;       // block size
    int64_t off;     // first column in the concatenated blocks
};

int counts_at(fl_op* op, const std::vector<double>& x, std::vector<int64_t>& c) {
    c.assign(x.size(), 0);
    if (x.empty()) return FL_OK;
    return fl_inertia_count(op, (int64_t)x.size(), x.data(), c.data(), nullptr);
}

// Nudges a point off an exact eigenvalue (a zero pivot gives count -1).
int robust_counts(fl_op* op, std::vector<double>& x, std::vector<int64_t>& c) {
    for (int tries = 0; tries < 4; ++tries) {
        int rc = counts_at(op, x, c);
        if (rc) return rc;
        bool bad = false;
        for (size_t k = 0; k < x.size(); ++k)
            if (c[k] < 0) {
                x[k] = x[k] * (1 + 1e-9) + 1e-300;
                bad = true;
            }
        if (!bad) return FL_OK;
    }
    return fl_fail(op->ctx, FL_ENOCONV, "spectrum slicing: a split point stays on an eigenvalue");
}

}  // namespace

extern "C" {

int fl_eigensolve_interval(fl_op* op, double lo, double hi, int64_t max_per_slice, double tol, int64_t cap,
                           double* theta, double* V, int64_t ldv, fl_slice_info* info) {
    if (!op) return FL_EINVAL;
    fl_ctx* ctx = op->ctx;
    if (info) *info = fl_slice_info{};
    if (!(lo < hi) || !std::isfinite(lo) || !std::isfinite(hi) || max_per_slice < 1 || max_per_slice > 500 ||
        cap < 0 || (cap > 0 && (!theta || !V || ldv < op->n)) || !(tol > 0.0 && tol < 1e-2))
        return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_interval: bad arguments");
    if (!op->rowptr) return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_interval: operator without a sparse pattern");
    FL_HIP(ctx, hipSetDevice(ctx->device));
    int rc = fl_inertia_prepare(op);
    if (rc) return rc;
    if (op->inert_bw > FL_BAND_MAX)
        return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_interval: bandwidth " + std::to_string(op->inert_bw) +
                                           " after reordering exceeds " + std::to_string(FL_BAND_MAX));
    const int64_t n = op->n;
    hipStream_t s = ctx->stream;
    // ---- 1. count
    std::vector<double> ends = {lo, hi};
    std::vector<int64_t> ce;
    if ((rc = robust_counts(op, ends, ce))) return rc;
    const double a0 = ends[0], b0 = ends[1];
    const int64_t m = ce[1] - ce[0];
    if (info) info->count = m;
    if (m > cap) return fl_fail(ctx, FL_EINVAL, "fl_eigensolve_interval: the interval holds " + std::to_string(m) +
                                                    " eigenvalues, more than cap = " + std::to_string(cap));
    if (m == 0) return FL_OK;
    // ---- 2. greedy partitioning
    int64_t S = (m + max_per_slice - 1) / max_per_slice;
    std::vector<double> pts(S + 1);  // split points, pts[0] = a0, pts[S] = b0
    std::vector<int64_t> cnt(S + 1);
    for (int64_t k = 0; k <= S; ++k) pts[k] = a0 + (b0 - a0) * (double)k / (double)S;
    cnt[0] = ce[0];
    cnt[S] = ce[1];
    std::vector<double> best_pts = pts;
    std::vector<int64_t> best_cnt;
    int64_t best_load = INT64_MAX;
    int rounds = 0;
    for (int round = 0; round < 7 && S > 1; ++round, ++rounds) {
        std::vector<double> inner(pts.begin() + 1, pts.end() - 1);
        std::vector<int64_t> ci;
        if ((rc = robust_counts(op, inner, ci))) return rc;
        for (int64_t k = 1; k < S; ++k) {
            pts[k] = inner[k - 1];
            cnt[k] = ci[k - 1];
        }
        int64_t load = 0;
        for (int64_t k = 0; k < S; ++k) load = std::max(load, cnt[k + 1] - cnt[k]);
        if (load < best_load) {
            best_load = load;
            best_pts = pts;
            best_cnt = cnt;
        }
        // new points: equal shares of the piecewise-linear cumulative count
        std::vector<double> np(pts);
        for (int64_t k = 1; k < S; ++k) {
            const double target = (double)ce[0] + (double)m * (double)k / (double)S;
            int64_t q = 0;
            while (q + 1 < S && (double)cnt[q + 1] < target) ++q;
            const double c0 = (double)cnt[q], c1 = (double)cnt[q + 1];
            const double f = c1 > c0 ? (target - c0) / (c1 - c0) : 0.5;
            np[k] = pts[q] + f * (pts[q + 1] - pts[q]);
        }
        for (int64_t k = 1; k < S; ++k) np[k] = std::max(np[k], np[k - 1]);
        pts = np;
    }
    if (S > 1) {
        pts = best_pts;
        cnt = best_cnt;
    }
    // slices above the limit are halved until none is
    for (int guard = 0; guard < 64; ++guard) {
        std::vector<double> mids;
        std::vector<int64_t> where;
        for (int64_t k = 0; k + 1 < (int64_t)pts.size(); ++k)
            if (cnt[k + 1] - cnt[k] > max_per_slice) {
                mids.push_back(0.5 * (pts[k] + pts[k + 1]));
                where.push_back(k);
            }
        if (mids.empty()) break;
        std::vector<int64_t> cm;
        if ((rc = robust_counts(op, mids, cm))) return rc;
        for (int64_t q = (int64_t)mids.size() - 1; q >= 0; --q) {
            pts.insert(pts.begin() + where[q] + 1, mids[q]);
            cnt.insert(cnt.begin() + where[q] + 1, cm[q]);
        }
    }
    std::vector<Slice> sl;
    int64_t ptot = 0;
    for (int64_t k = 0; k + 1 < (int64_t)pts.size(); ++k) {
        const int64_t mk = cnt[k + 1] - cnt[k];
        if (mk > max_per_slice) return fl_fail(ctx, FL_ENOCONV, "spectrum slicing: partitioning did not converge");
        if (mk == 0) continue;
        Slice q{pts[k], pts[k + 1], mk, std::min<int64_t>(std::min<int64_t>(2 * mk + 16, 1024), n), ptot};
        sl.push_back(q);
        ptot += q.p;
    }
    const int64_t ns = (int64_t)sl.size();
    if (info) {
        info->slices = ns;
        info->partition_rounds = rounds;
        info->max_load = 0;
        for (const Slice& q : sl) info->max_load = std::max(info->max_load, q.m);
    }
    // ---- 3. factor every shifted pencil, then subspace iteration
    const int64_t bw = std::max<int64_t>(op->inert_bw, 1);
    const int64_t ldb = fl_band_ldb(bw), stride = fl_band_stride(n, bw);
    DevBuf bband, blrow, bsig, bneg, bX, bKY, bMY, bKp, bMp, bZ, bth, blt, brel, bprobs, bss, bbs, bbc, bscale, bcs;
    FL_HIP(ctx, bband.alloc((size_t)(ns * stride) * 8));
    FL_HIP(ctx, blrow.alloc((size_t)(ns * stride) * 8));
    FL_HIP(ctx, bsig.alloc(ns * 8));
    FL_HIP(ctx, bneg.alloc(ns * 8));
    std::vector<double> sig(ns);
    for (int64_t k = 0; k < ns; ++k) sig[k] = 0.5 * (sl[k].a + sl[k].b);
    FL_HIP(ctx, hipMemcpyAsync(bsig.p, sig.data(), ns * 8, hipMemcpyHostToDevice, s));
    FL_HIP(ctx, fl_band_factor(s, op, ns, bsig.as<double>(), bband.as<double>(), blrow.as<double>(),
                               bneg.as<int64_t>()));
    {
        std::vector<int64_t> neg(ns);
        FL_HIP(ctx, hipMemcpyAsync(neg.data(), bneg.p, ns * 8, hipMemcpyDeviceToHost, s));
        FL_HIP(ctx, hipStreamSynchronize(s));
        for (int64_t k = 0; k < ns; ++k)
            if (neg[k] < 0) return fl_fail(ctx, FL_ENOCONV, "spectrum slicing: a slice shift is an eigenvalue");
    }
    const size_t nX = (size_t)n * ptot;
    DevBuf bT, bY;
    FL_HIP(ctx, bX.alloc(nX * 8));
    FL_HIP(ctx, bT.alloc(nX * 8));
    FL_HIP(ctx, bY.alloc(nX * 8));
    FL_HIP(ctx, bKY.alloc(nX * 8));
    FL_HIP(ctx, bMY.alloc(nX * 8));
    int64_t pp = 0;  // sum of p_s^2
    for (const Slice& q : sl) pp += q.p * q.p;
    FL_HIP(ctx, bKp.alloc(pp * 8));
    FL_HIP(ctx, bMp.alloc(pp * 8));
    FL_HIP(ctx, bZ.alloc(pp * 8));
    FL_HIP(ctx, bth.alloc(ptot * 8));
    FL_HIP(ctx, blt.alloc(ptot * 8));
    FL_HIP(ctx, brel.alloc(ptot * 8));
    FL_HIP(ctx, bscale.alloc(ptot * 8));
    FL_HIP(ctx, bcs.alloc(ptot * 8));
    {
        std::vector<double> sc(ptot), cs(ptot);
        for (int64_t k = 0; k < ns; ++k)
            for (int64_t j = 0; j < sl[k].p; ++j) {
                sc[sl[k].off + j] = std::fabs(sl[k].b);
                cs[sl[k].off + j] = sig[k];
            }
        FL_HIP(ctx, hipMemcpyAsync(bscale.p, sc.data(), ptot * 8, hipMemcpyHostToDevice, s));
        FL_HIP(ctx, hipMemcpyAsync(bcs.p, cs.data(), ptot * 8, hipMemcpyHostToDevice, s));
        FL_HIP(ctx, hipStreamSynchronize(s));
    }
    double* X = bX.as<double>();    // current block (natural numbering)
    double* T = bT.as<double>();    // solves (banded numbering); K X afterwards
    double* Y = bY.as<double>();    // (K - sigma M)^-1 M X; M X afterwards
    double* KY = bKY.as<double>();
    double* MY = bMY.as<double>();
    // per-slice solve descriptors and the block -> (slice, column) map
    std::vector<SliceSolve> hs(ns);
    std::vector<int> blk_slice, blk_col;
    for (int64_t k = 0; k < ns; ++k) {
        hs[k] = SliceSolve{bband.as<double>() + k * stride, blrow.as<double>() + k * stride, T + sl[k].off * n,
                           (int)sl[k].p};
        for (int64_t c0 = 0; c0 < sl[k].p; c0 += SOLVE_COLS) {
            blk_slice.push_back((int)k);
            blk_col.push_back((int)c0);
        }
    }
    FL_HIP(ctx, bss.alloc(sizeof(SliceSolve) * ns));
    FL_HIP(ctx, bbs.alloc(sizeof(int) * blk_slice.size()));
    FL_HIP(ctx, bbc.alloc(sizeof(int) * blk_col.size()));
    FL_HIP(ctx, hipMemcpyAsync(bss.p, hs.data(), sizeof(SliceSolve) * ns, hipMemcpyHostToDevice, s));
    FL_HIP(ctx, hipMemcpyAsync(bbs.p, blk_slice.data(), sizeof(int) * blk_slice.size(), hipMemcpyHostToDevice, s));
    FL_HIP(ctx, hipMemcpyAsync(bbc.p, blk_col.data(), sizeof(int) * blk_col.size(), hipMemcpyHostToDevice, s));
    // batched products, five groups of ns:
    //   Kp = Y^T (K Y), Mp = Y^T (M Y), X = Y Z, T = (K Y) Z = K X, Y = (M Y) Z = M X
    std::vector<int64_t> zo(ns);
    {
        int64_t zoff = 0;
        for (int64_t k = 0; k < ns; ++k) {
            zo[k] = zoff;
            zoff += sl[k].p * sl[k].p;
        }
    }
    std::vector<GemmProblem> gp;
    auto add_proj = [&](const double* B, double* C) {
        for (int64_t k = 0; k < ns; ++k) {
            const int64_t p = sl[k].p;
            gp.push_back(GemmProblem{p, p, n, Y + sl[k].off * n, n, B + sl[k].off * n, n, C + zo[k], p, 1.0, 0.0});
        }
    };
    auto add_rot = [&](const double* A, double* C) {
        for (int64_t k = 0; k < ns; ++k) {
            const int64_t p = sl[k].p;
            gp.push_back(GemmProblem{n, p, p, A + sl[k].off * n, n, bZ.as<double>() + zo[k], p, C + sl[k].off * n, n,
                                     1.0, 0.0});
        }
    };
    add_proj(KY, bKp.as<double>());
    add_proj(MY, bMp.as<double>());
    add_rot(Y, X);
    add_rot(KY, T);
    add_rot(MY, Y);
    FL_HIP(ctx, bprobs.alloc(sizeof(GemmProblem) * gp.size()));
    FL_HIP(ctx, hipMemcpyAsync(bprobs.p, gp.data(), sizeof(GemmProblem) * gp.size(), hipMemcpyHostToDevice, s));
    const GemmProblem* dprobs = bprobs.as<GemmProblem>();
    int64_t pmax = 0;
    for (const Slice& q : sl) pmax = std::max(pmax, q.p);
    // operators of the projected pencils for the batched eigensolver
    std::vector<fl_op> pops(ns);
    std::vector<fl_op*> pptr(ns);
    for (int64_t k = 0; k < ns; ++k) {
        fl_op& o = pops[k];
        o.ctx = ctx;
        o.device = ctx->device;
        o.n = sl[k].p;
        o.ld = sl[k].p;
        o.K = bKp.as<double>() + zo[k];
        o.M = bMp.as<double>() + zo[k];
        o.V = bZ.as<double>() + zo[k];
        o.theta = bth.as<double>() + sl[k].off;
        o.logtheta = blt.as<double>() + sl[k].off;
        pptr[k] = &o;
    }
    auto release_pops = [&]() {
        for (fl_op& o : pops) o.K = o.M = o.V = o.theta = o.logtheta = nullptr;
    };
    start_block_kernel<<<1024, 256, 0, s>>>((int64_t)nX, 0x2545F4914F6CDD1Dull, X);
    FL_HIP(ctx, hipGetLastError());
    const dim3 pg((unsigned)FL_DIV_UP(n, 256), (unsigned)std::min<int64_t>(ptot, 65535));
    const dim3 rg((unsigned)FL_DIV_UP(n, 256), (unsigned)std::min<int64_t>(FL_DIV_UP(ptot, RES_COLS), 65535));
    std::vector<double> th(ptot), rel(ptot);
    int it = 0;
    double worst = 0.0;
    const int MAX_IT = 200;
    for (; it < MAX_IT; ++it) {
        // Y = (K - sigma_s M)^-1 M X, the solves in the banded numbering,
        // then one step of iterative refinement: R = M X - (K - sigma_s M) Y
        // (into X, which M X has replaced), Y += (K - sigma_s M)^-1 R
        FL_HIP(ctx, fl_spmm_csr(s, n, op->rowptr, op->colidx, op->mval, ptot, X, n, KY, n));
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1) {
                shifted_residual_kernel<<<rg, 256, 0, s>>>(n, op->rowptr, op->colidx, op->kval, op->mval, ptot,
                                                           bcs.as<double>(), KY, Y, X);
                FL_HIP(ctx, hipGetLastError());
            }
            permute_rows_kernel<<<pg, 256, 0, s>>>(n, ptot, op->inert_pinv, pass ? X : KY, T, TO_BAND);
            FL_HIP(ctx, hipGetLastError());
            band_solve_kernel<<<(unsigned)blk_slice.size(), 64, 0, s>>>(n, (int)bw, ldb, bss.as<SliceSolve>(),
                                                                        bbs.as<int>(), bbc.as<int>());
            FL_HIP(ctx, hipGetLastError());
            permute_rows_kernel<<<pg, 256, 0, s>>>(n, ptot, op->inert_pinv, T, Y, pass ? ADD_FROM_BAND : FROM_BAND);
            FL_HIP(ctx, hipGetLastError());
        }
        // Rayleigh-Ritz per slice on M-normalised columns
        FL_HIP(ctx, fl_spmm_csr(s, n, op->rowptr, op->colidx, op->kval, ptot, Y, n, KY, n));
        FL_HIP(ctx, fl_spmm_csr(s, n, op->rowptr, op->colidx, op->mval, ptot, Y, n, MY, n));
        mnormalise_kernel<<<(unsigned)ptot, 256, 0, s>>>(n, Y, KY, MY);
        FL_HIP(ctx, hipGetLastError());
        FL_HIP(ctx, fl_dgemm_batched(s, 1, 0, dprobs, (int)(2 * ns), pmax, pmax));
        rc = fl_eigensolve_batched(ctx, ns, pptr.data(), FL_FP64, nullptr);
        if (rc) {
            release_pops();
            return fl_fail(ctx, rc, std::string("spectrum slicing: Rayleigh-Ritz: ") + ctx->err);
        }
        FL_HIP(ctx, fl_dgemm_batched(s, 0, 0, dprobs + 2 * ns, (int)ns, n, pmax));  // X = Y Z
        FL_HIP(ctx, fl_dgemm_batched(s, 0, 0, dprobs + 3 * ns, (int)ns, n, pmax));  // T = K X
        FL_HIP(ctx, fl_dgemm_batched(s, 0, 0, dprobs + 4 * ns, (int)ns, n, pmax));  // Y = M X
        ritz_residual_kernel<<<(unsigned)ptot, 256, 0, s>>>(n, T, Y, bth.as<double>(), bscale.as<double>(),
                                                             brel.as<double>());
        FL_HIP(ctx, hipGetLastError());
        FL_HIP(ctx, hipMemcpyAsync(th.data(), bth.p, ptot * 8, hipMemcpyDeviceToHost, s));
        FL_HIP(ctx, hipMemcpyAsync(rel.data(), brel.p, ptot * 8, hipMemcpyDeviceToHost, s));
        FL_HIP(ctx, hipStreamSynchronize(s));
        // converged Ritz pairs inside each slice (unconverged Ritz values of the
        // guard directions are mixtures and may fall anywhere); a slice is
        // done when they number exactly its inertia count
        bool all = true;
        worst = 0.0;
        for (int64_t k = 0; k < ns; ++k) {
            int64_t good = 0;
            double w = 0.0;
            for (int64_t j = 0; j < sl[k].p; ++j) {
                const double t = th[sl[k].off + j], r = rel[sl[k].off + j];
                if (t >= sl[k].a && t < sl[k].b && r <= tol) {
                    ++good;
                    w = std::max(w, r);
                }
            }
            worst = std::max(worst, good == sl[k].m ? w : 1.0);
            all = all && good == sl[k].m;
        }
        if (all) break;
    }
    release_pops();
    if (info) {
        info->iterations = it + 1;
        info->max_residual = worst;
    }
    if (it == MAX_IT) return fl_fail(ctx, FL_ENOCONV, "spectrum slicing: subspace iteration did not converge");
    // ---- 4. the pairs inside each slice, in slice order (ascending)
    std::vector<int64_t> idx;
    for (int64_t k = 0; k < ns; ++k)
        for (int64_t j = 0; j < sl[k].p; ++j) {
            const double t = th[sl[k].off + j];
            if (t >= sl[k].a && t < sl[k].b && rel[sl[k].off + j] <= tol) idx.push_back(sl[k].off + j);
        }
    if ((int64_t)idx.size() != m) return fl_fail(ctx, FL_ENOCONV, "spectrum slicing: pairs lost in post-processing");
    DevBuf bidx;
    FL_HIP(ctx, bidx.alloc(sizeof(int64_t) * m));
    FL_HIP(ctx, hipMemcpyAsync(bidx.p, idx.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, s));
    gather_pairs_kernel<<<dim3((unsigned)std::min<int64_t>(FL_DIV_UP(n, 256), 64),
                               (unsigned)std::min<int64_t>(m, 65535)), 256, 0, s>>>(n, m, bidx.as<int64_t>(), X,
                                                                                    bth.as<double>(), V, ldv, theta);
    FL_HIP(ctx, hipGetLastError());
    // post-processing: one Newton-Schulz step V := V (3 I - V^T M V) / 2 makes
    // the columns M-orthonormal across slices to second order (within a slice
    // they already are; across slices their products are of the size of the
    // residuals over the gaps); the eigenvalues stay the Ritz values
    {
        DevBuf bG;
        FL_HIP(ctx, bG.alloc((size_t)m * m * 8));
        double* G = bG.as<double>();
        FL_HIP(ctx, fl_spmm_csr(s, n, op->rowptr, op->colidx, op->mval, m, V, ldv, KY, n));
        FL_HIP(ctx, fl_dgemm(s, 1, 0, m, m, n, 1.0, V, ldv, KY, n, 0.0, G, m));
        newton_schulz_kernel<<<dim3((unsigned)FL_DIV_UP(m, 256), (unsigned)std::min<int64_t>(m, 65535)), 256, 0, s>>>(
            m, G);
        FL_HIP(ctx, hipGetLastError());
        FL_HIP(ctx, fl_dgemm(s, 0, 0, n, m, m, 1.0, V, ldv, G, m, 0.0, T, n));
        FL_HIP(ctx, fl_copy_matrix(s, n, m, T, n, V, ldv));
        FL_HIP(ctx, hipStreamSynchronize(s));
    }
    return FL_OK;
}

}  // extern "C"
