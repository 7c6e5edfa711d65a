// Input stage: Galerkin stiffness and mass matrices (eq. discrete_laplace,
// K_ij = <grad e_i, grad e_j>, M_ij = <e_i, e_j>) assembled on the GPU.
//
// Element matrices in closed form:
//  * bilinear element on an axis-aligned hx x hy rectangle: tensor products
//    of the 1-D linear-element matrices k = (1/h)[[1,-1],[-1,1]] and
//    m = (h/6)[[2,1],[1,2]]:  Ke = kx (x) my + mx (x) ky,  Me = mx (x) my;
//  * linear triangle of area A with barycentric gradients g_i:
//    Ke_ij = A g_i . g_j,  Me_ij = (A/12)(1 + delta_ij).
// Elements arrive grouped by colour (no two elements of a colour share a
// node), so the scatter-add into the dense matrices needs no atomics and the
// result is bitwise reproducible.
#include "internal.h"

namespace {

template <int NV>
__global__ void assemble_kernel(const double* __restrict__ xy, const int32_t* __restrict__ conn, int64_t e0,
                                int64_t e1, const int64_t* __restrict__ dof, int64_t ld, double* K, double* M) {
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
            K[g[a] + g[b] * ld] += Ke[a][b];
            M[g[a] + g[b] * ld] += Me[a][b];
        }
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

hipError_t fl_assemble_launch(hipStream_t s, int elem, const double* xy, const int32_t* conn_sorted,
                              const int64_t* color_start, int ncolor, const int64_t* dof, int64_t n, int64_t ld,
                              double* K, double* M) {
    for (int c = 0; c < ncolor; ++c) {
        int64_t e0 = color_start[c], e1 = color_start[c + 1];
        if (e1 <= e0) continue;
        unsigned blocks = (unsigned)FL_DIV_UP(e1 - e0, 128);
        if (elem == 4)
            assemble_kernel<4><<<blocks, 128, 0, s>>>(xy, conn_sorted, e0, e1, dof, ld, K, M);
        else
            assemble_kernel<3><<<blocks, 128, 0, s>>>(xy, conn_sorted, e0, e1, dof, ld, K, M);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t fl_csr_gather(hipStream_t s, int64_t n, const int32_t* rowptr, const int32_t* colidx, const double* K,
                         const double* M, int64_t ld, double* kval, double* mval) {
    if (n <= 0) return hipSuccess;
    csr_gather_kernel<<<(unsigned)FL_DIV_UP(n, 256), 256, 0, s>>>(n, rowptr, colidx, K, M, ld, kval, mval);
    return hipGetLastError();
}
