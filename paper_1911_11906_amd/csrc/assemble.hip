// Input stage: Galerkin stiffness and mass matrices (eq. discrete_laplace,
// K_ij = <grad e_i, grad e_j>, M_ij = <e_i, e_j>) assembled on the GPU.
//
// Element matrices in closed form:
//  * bilinear element on an axis-aligned hx x hy rectangle: tensor products
//    of the 1-D linear-element matrices k = (1/h)[[1,-1],[-1,1]] and
//    m = (h/6)[[2,1],[1,2]]:  Ke = kx (x) my + mx (x) ky,  Me = mx (x) my;
//  * linear triangle of area A with barycentric gradients g_i:
//    Ke_ij = A g_i . g_j,  Me_ij = (A/12)(1 + delta_ij);
//  * tensor-product element of order p = 2..8 on an axis-aligned rectangle
//    ((p+1)^2 nodes, lexicographic a + (p+1) b): the same tensor-product form
//    with the 1-D order-p matrices k_ac = int l_a' l_c' and m_ac = int l_a l_c
//    of the Lagrange basis through the element's node positions, integrated
//    by the (p+1)-point Gauss rule (exact for degree 2p + 1) computed in the
//    kernel; one workgroup per element.
// Elements arrive grouped by colour (no two elements of a colour share a
// node), so the scatter-add needs no atomics and the result is bitwise
// reproducible.  The contributions go into dense K and M, or (for pencils
// too large for dense storage) straight into the values of the CSR pattern.
#include "internal.h"

namespace {

// Where element contributions go: dense column-major K, M, or the values of
// the CSR pattern (entry (i, j) found by a binary search of row i's sorted
// column indices).
struct DenseSink {
    double* K;
    double* M;
    int64_t ld;
    __device__ inline void add(int64_t i, int64_t j, double k, double m) const {
        K[i + j * ld] += k;
        M[i + j * ld] += m;
    }
};
struct CsrSink {
    const int32_t* rowptr;
    const int32_t* colidx;
    double* kval;
    double* mval;
    __device__ inline void add(int64_t i, int64_t j, double k, double m) const {
        int32_t lo = rowptr[i], hi = rowptr[i + 1] - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (colidx[mid] < j) lo = mid + 1;
            else hi = mid;
        }
        kval[lo] += k;
        mval[lo] += m;
    }
};

template <int NV, class Sink>
__global__ void assemble_kernel(const double* __restrict__ xy, const int32_t* __restrict__ conn, int64_t e0,
                                int64_t e1, const int64_t* __restrict__ dof, Sink sink) {
    int64_t e = e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= e1) return;
    double x[NV], y[NV];
    int64_t g[NV];
#pragma unroll
    for (int a = 0; a < NV; ++a) {
        int32_t v = conn[e * NV + a];
        x[a] = xy[2 * (int64_t)v];
        y[a] = xy[2 * (int64_t)v + 1];
        g[a] = dof[v];
    }
    double Ke[NV][NV], Me[NV][NV];
    if (NV == 4) {
        double xmin = fmin(fmin(x[0], x[1]), fmin(x[2], x[3])), xmax = fmax(fmax(x[0], x[1]), fmax(x[2], x[3]));
        double ymin = fmin(fmin(y[0], y[1]), fmin(y[2], y[3])), ymax = fmax(fmax(y[0], y[1]), fmax(y[2], y[3]));
        double hx = xmax - xmin, hy = ymax - ymin;
        int sx[NV], sy[NV];
#pragma unroll
        for (int a = 0; a < NV; ++a) {
            sx[a] = (x[a] == xmax) ? 1 : 0;
            sy[a] = (y[a] == ymax) ? 1 : 0;
        }
#pragma unroll
        for (int a = 0; a < NV; ++a)
#pragma unroll
            for (int b = 0; b < NV; ++b) {
                double kx = (sx[a] == sx[b] ? 1.0 : -1.0) / hx, ky = (sy[a] == sy[b] ? 1.0 : -1.0) / hy;
                double mx = (sx[a] == sx[b] ? 2.0 : 1.0) * hx / 6.0, my = (sy[a] == sy[b] ? 2.0 : 1.0) * hy / 6.0;
                Ke[a][b] = kx * my + mx * ky;
                Me[a][b] = mx * my;
            }
    } else {
        double det = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
        double area = 0.5 * det;
        double bx[NV], by[NV];
#pragma unroll
        for (int a = 0; a < NV; ++a) {
            int p = (a + 1) % 3, q = (a + 2) % 3;
            bx[a] = (y[p] - y[q]) / det;
            by[a] = (x[q] - x[p]) / det;
        }
#pragma unroll
        for (int a = 0; a < NV; ++a)
#pragma unroll
            for (int b = 0; b < NV; ++b) {
                Ke[a][b] = area * (bx[a] * bx[b] + by[a] * by[b]);
                Me[a][b] = (a == b ? 2.0 : 1.0) * area / 12.0;
            }
    }
#pragma unroll
    for (int a = 0; a < NV; ++a) {
        if (g[a] < 0) continue;
#pragma unroll
        for (int b = 0; b < NV; ++b) {
            if (g[b] < 0) continue;
            sink.add(g[a], g[b], Ke[a][b], Me[a][b]);
        }
    }
}

// Nodes and weights of the Q-point Gauss-Legendre rule: thread i < Q finds
// root i of P_Q by Newton's method (P_Q and P_Q' by the three-term
// recurrence) from the estimate cos(pi (i + 3/4) / (Q + 1/2)).
template <int Q>
__device__ void gauss_rule(double* gp, double* gw) {
    const int i = threadIdx.x;
    if (i >= Q) return;
    double z = cos(3.141592653589793 * (i + 0.75) / (Q + 0.5)), dpq = 1.0;
    for (int it = 0; it < 60; ++it) {
        double pm = 1.0, pq = z;  // P_{k-1}, P_k
        for (int k = 1; k < Q; ++k) {
            const double pn = ((2 * k + 1) * z * pq - k * pm) / (k + 1);
            pm = pq;
            pq = pn;
        }
        dpq = Q * (z * pq - pm) / (z * z - 1.0);
        const double dz = pq / dpq;
        z -= dz;
        if (fabs(dz) <= 1e-16) break;
    }
    gp[i] = z;
    gw[i] = 2.0 / ((1.0 - z * z) * dpq * dpq);
}

template <int P, class Sink>
__global__ __launch_bounds__(256) void assemble_qp_kernel(const double* __restrict__ xy, const int32_t* __restrict__ conn,
                                                          int64_t e0, const int64_t* __restrict__ dof, Sink sink) {
    constexpr int Q = P + 1, NV = Q * Q;
    __shared__ double gp[Q], gw[Q], sx[Q], sy[Q], box[4];
    __shared__ double Lx[Q][Q], Dx[Q][Q], Ly[Q][Q], Dy[Q][Q];  // [quadrature point][basis function]
    __shared__ double kx[Q][Q], mx[Q][Q], ky[Q][Q], my[Q][Q];
    __shared__ int64_t g[NV];
    const int64_t e = e0 + blockIdx.x;
    const int t = threadIdx.x;
    const int32_t* cn = conn + e * NV;
    if (t < NV) g[t] = dof[cn[t]];
    if (t == 0) {
        box[0] = xy[2 * (int64_t)cn[0]];
        box[1] = xy[2 * (int64_t)cn[P]];
        box[2] = xy[2 * (int64_t)cn[0] + 1];
        box[3] = xy[2 * (int64_t)cn[P * Q] + 1];
    }
    gauss_rule<Q>(gp, gw);
    __syncthreads();
    const double hx = box[1] - box[0], hy = box[3] - box[2];
    if (t < Q) {
        sx[t] = -1.0 + 2.0 * (xy[2 * (int64_t)cn[t]] - box[0]) / hx;
        sy[t] = -1.0 + 2.0 * (xy[2 * (int64_t)cn[t * Q] + 1] - box[2]) / hy;
    }
    __syncthreads();
    // Lagrange basis function a (and its derivative) at quadrature point q
    if (t < 2 * Q * Q) {
        const int dir = t / (Q * Q), q = (t % (Q * Q)) / Q, a = t % Q;
        const double* s = dir ? sy : sx;
        const double z = gp[q];
        double v = 1.0, d = 0.0;
        for (int b = 0; b < Q; ++b) {
            if (b == a) continue;
            const double f = (z - s[b]) / (s[a] - s[b]);
            d = d * f + v / (s[a] - s[b]);
            v *= f;
        }
        if (dir) {
            Ly[q][a] = v;
            Dy[q][a] = d;
        } else {
            Lx[q][a] = v;
            Dx[q][a] = d;
        }
    }
    __syncthreads();
    // 1-D element matrices (reference interval [-1, 1] of length h / 2 per unit)
    if (t < 2 * Q * Q) {
        const int dir = t / (Q * Q), a = (t % (Q * Q)) / Q, c = t % Q;
        const double h = dir ? hy : hx;
        double kk = 0.0, mm = 0.0;
        for (int q = 0; q < Q; ++q) {
            if (dir) {
                kk += gw[q] * Dy[q][a] * Dy[q][c];
                mm += gw[q] * Ly[q][a] * Ly[q][c];
            } else {
                kk += gw[q] * Dx[q][a] * Dx[q][c];
                mm += gw[q] * Lx[q][a] * Lx[q][c];
            }
        }
        if (dir) {
            ky[a][c] = (2.0 / h) * kk;
            my[a][c] = 0.5 * h * mm;
        } else {
            kx[a][c] = (2.0 / h) * kk;
            mx[a][c] = 0.5 * h * mm;
        }
    }
    __syncthreads();
    for (int idx = t; idx < NV * NV; idx += 256) {
        const int i = idx % NV, j = idx / NV;
        const int64_t gi = g[i], gj = g[j];
        if (gi < 0 || gj < 0) continue;
        const int a = i % Q, b = i / Q, c = j % Q, d = j / Q;
        sink.add(gi, gj, kx[a][c] * my[b][d] + mx[a][c] * ky[b][d], mx[a][c] * my[b][d]);
    }
}

__global__ void csr_gather_kernel(int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                                  const double* __restrict__ K, const double* __restrict__ M, int64_t ld,
                                  double* kval, double* mval) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        int64_t j = colidx[p];
        kval[p] = K[i + j * ld];
        mval[p] = M[i + j * ld];
    }
}

}  // namespace

namespace {
template <class Sink>
hipError_t assemble_colours(hipStream_t s, int elem, const double* xy, const int32_t* conn_sorted,
                            const int64_t* color_start, int ncolor, const int64_t* dof, const Sink& sink) {
    for (int c = 0; c < ncolor; ++c) {
        int64_t e0 = color_start[c], e1 = color_start[c + 1];
        if (e1 <= e0) continue;
        unsigned blocks = (unsigned)FL_DIV_UP(e1 - e0, 128);
        const unsigned eb = (unsigned)(e1 - e0);
        switch (elem) {
            case 3: assemble_kernel<3><<<blocks, 128, 0, s>>>(xy, conn_sorted, e0, e1, dof, sink); break;
            case 4: assemble_kernel<4><<<blocks, 128, 0, s>>>(xy, conn_sorted, e0, e1, dof, sink); break;
            case 9: assemble_qp_kernel<2><<<eb, 256, 0, s>>>(xy, conn_sorted, e0, dof, sink); break;
            case 16: assemble_qp_kernel<3><<<eb, 256, 0, s>>>(xy, conn_sorted, e0, dof, sink); break;
            case 25: assemble_qp_kernel<4><<<eb, 256, 0, s>>>(xy, conn_sorted, e0, dof, sink); break;
            case 36: assemble_qp_kernel<5><<<eb, 256, 0, s>>>(xy, conn_sorted, e0, dof, sink); break;
            case 49: assemble_qp_kernel<6><<<eb, 256, 0, s>>>(xy, conn_sorted, e0, dof, sink); break;
            case 64: assemble_qp_kernel<7><<<eb, 256, 0, s>>>(xy, conn_sorted, e0, dof, sink); break;
            case 81: assemble_qp_kernel<8><<<eb, 256, 0, s>>>(xy, conn_sorted, e0, dof, sink); break;
            default: return hipErrorInvalidValue;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
}  // namespace

hipError_t fl_assemble_launch(hipStream_t s, int elem, const double* xy, const int32_t* conn_sorted,
                              const int64_t* color_start, int ncolor, const int64_t* dof, int64_t n, int64_t ld,
                              double* K, double* M) {
    return assemble_colours(s, elem, xy, conn_sorted, color_start, ncolor, dof, DenseSink{K, M, ld});
}

hipError_t fl_assemble_csr_launch(hipStream_t s, int elem, const double* xy, const int32_t* conn_sorted,
                                  const int64_t* color_start, int ncolor, const int64_t* dof, const int32_t* rowptr,
                                  const int32_t* colidx, double* kval, double* mval) {
    return assemble_colours(s, elem, xy, conn_sorted, color_start, ncolor, dof,
                            CsrSink{rowptr, colidx, kval, mval});
}

hipError_t fl_csr_gather(hipStream_t s, int64_t n, const int32_t* rowptr, const int32_t* colidx, const double* K,
                         const double* M, int64_t ld, double* kval, double* mval) {
    if (n <= 0) return hipSuccess;
    csr_gather_kernel<<<(unsigned)FL_DIV_UP(n, 256), 256, 0, s>>>(n, rowptr, colidx, K, M, ld, kval, mval);
    return hipGetLastError();
}
