/*
 * Plain FP64 CPU oracle for the eigenfunction-expansion fractional Poisson
 * solver (Carlson, Kirby, Sundar, "A Scalable Framework for Solving
 * Fractional Diffusion Equations").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU library.
 *
 * What it computes, step by step, is the definition written out:
 *   - the Galerkin pencil K_ij = <grad e_i, grad e_j>, M_ij = <e_i, e_j>
 *     (Section "Method", equation discrete_laplace and the definition of K and M
 *     below it), element integrals by Gauss quadrature that is exact for the
 *     integrands (bilinear quads: 2x2 Gauss; linear triangles: edge-midpoint
 *     rule for the mass, constant gradients for the stiffness);
 *     homogeneous Dirichlet nodes are eliminated (Section "Accuracy");
 *   - all n pairs K phi = theta M phi with phi_j^T M phi_k = delta_jk
 *     (equation discrete_laplace; orthonormality from Section
 *     "Post-processing"), via M = L L^T, C = L^-1 K L^-T, cyclic two-sided
 *     Jacobi on C (parallel round-robin order), phi = L^-T q;
 *   - the discrete solution v = sum_k theta_k^(-alpha/2) <f, phi_k> phi_k with
 *     <f, phi_k> = phi_k^T M f (the equation for g and v in Section "Method");
 *   - its adjoint with respect to f and alpha;
 *   - the solution of the fractional diffusion equation
 *     u(t) = sum_k exp(-mu theta_k^(alpha/2) t) <u0, phi_k> phi_k (equation
 *     diffusion_solution) and its adjoint with respect to u0, alpha, t, mu.
 *
 * Elements: linear triangles, bilinear quadrilaterals and, for the order
 * sweep of Section "Accuracy", tensor-product Lagrange elements of order
 * p = 2..8 on axis-aligned rectangles ((p+1)^2 nodes, lexicographic).
 *
 * All matrices are column-major: A[i + j*lda].
 * Precision: IEEE double throughout.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Element matrices by quadrature                                            */
/* ------------------------------------------------------------------------ */

/* Bilinear quadrilateral (isoparametric map from [-1,1]^2), nodes CCW:
 * (-1,-1), (1,-1), (1,1), (-1,1).  2x2 Gauss points integrate the
 * stiffness and mass integrands exactly when the element is a parallelogram. */
static int q1_element(const double *x, const double *y, double Ke[16], double Me[16]) {
    static const double sx[4] = {-1.0, 1.0, 1.0, -1.0};
    static const double sy[4] = {-1.0, -1.0, 1.0, 1.0};
    const double g = 1.0 / sqrt(3.0);
    const double gp[2] = {-g, g};
    memset(Ke, 0, 16 * sizeof(double));
    memset(Me, 0, 16 * sizeof(double));
    for (int a = 0; a < 2; ++a) {
        for (int b = 0; b < 2; ++b) {
            double xi = gp[a], eta = gp[b];
            double N[4], dNxi[4], dNeta[4];
            for (int k = 0; k < 4; ++k) {
                N[k] = 0.25 * (1.0 + sx[k] * xi) * (1.0 + sy[k] * eta);
                dNxi[k] = 0.25 * sx[k] * (1.0 + sy[k] * eta);
                dNeta[k] = 0.25 * sy[k] * (1.0 + sx[k] * xi);
            }
            double J11 = 0, J12 = 0, J21 = 0, J22 = 0; /* J = d(x,y)/d(xi,eta) */
            for (int k = 0; k < 4; ++k) {
                J11 += dNxi[k] * x[k];
                J12 += dNxi[k] * y[k];
                J21 += dNeta[k] * x[k];
                J22 += dNeta[k] * y[k];
            }
            double det = J11 * J22 - J12 * J21;
            if (!(det > 0.0)) return -1;
            double dNx[4], dNy[4];
            for (int k = 0; k < 4; ++k) {
                /* [dN/dx; dN/dy] = J^{-1} [dN/dxi; dN/deta] */
                dNx[k] = (J22 * dNxi[k] - J12 * dNeta[k]) / det;
                dNy[k] = (-J21 * dNxi[k] + J11 * dNeta[k]) / det;
            }
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    Ke[i * 4 + j] += det * (dNx[i] * dNx[j] + dNy[i] * dNy[j]);
                    Me[i * 4 + j] += det * N[i] * N[j];
                }
        }
    }
    return 0;
}

/* Linear triangle: constant gradients; the mass integrand is quadratic and
 * the three-edge-midpoint rule (weights area/3) integrates it exactly. */
static int p1_element(const double *x, const double *y, double Ke[9], double Me[9]) {
    double det = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
    if (!(det > 0.0)) return -1;
    double area = 0.5 * det;
    /* barycentric gradients: grad lambda_i = (y_j - y_k, x_k - x_j) / det */
    double gx[3], gy[3];
    for (int i = 0; i < 3; ++i) {
        int j = (i + 1) % 3, k = (i + 2) % 3;
        gx[i] = (y[j] - y[k]) / det;
        gy[i] = (x[k] - x[j]) / det;
    }
    /* barycentric coordinates of the edge midpoints */
    static const double mid[3][3] = {{0.5, 0.5, 0.0}, {0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            Ke[i * 3 + j] = area * (gx[i] * gx[j] + gy[i] * gy[j]);
            double m = 0.0;
            for (int q = 0; q < 3; ++q) m += (area / 3.0) * mid[q][i] * mid[q][j];
            Me[i * 3 + j] = m;
        }
    return 0;
}

/* Gauss-Legendre rule with m points on [-1, 1]: the nodes are the roots of
 * the Legendre polynomial P_m, found by Newton's method from the estimates
 * cos(pi (i + 3/4) / (m + 1/2)), with P_m and P_m' from the three-term
 * recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}; the weights are
 * 2 / ((1 - x^2) P_m'(x)^2).  Exact for polynomials of degree 2m - 1. */
static void gauss_legendre(int m, double *x, double *w) {
    for (int i = 0; i < m; ++i) {
        double z = cos(acos(-1.0) * (i + 0.75) / (m + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 1; k < m; ++k) {
                double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            /* P_m = p1, P_{m-1} = p0; P_m' = m (z P_m - P_{m-1}) / (z^2 - 1) */
            dp = m * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Lagrange basis through the nodes s[0..p] at t: values L[a] and
 * derivatives D[a] (product rule over the factors (t - s_b)/(s_a - s_b)). */
static void lagrange_basis(int p, const double *s, double t, double *L, double *D) {
    for (int a = 0; a <= p; ++a) {
        double v = 1.0, d = 0.0;
        for (int b = 0; b <= p; ++b) {
            if (b == a) continue;
            double f = (t - s[b]) / (s[a] - s[b]);
            d = d * f + v / (s[a] - s[b]);
            v *= f;
        }
        L[a] = v;
        D[a] = d;
    }
}

/* Tensor-product element of order p on an axis-aligned rectangle, nodes in
 * lexicographic order a + (p+1) b (a along x).  The reference coordinates
 * of the nodes follow from the physical ones (bottom row for x, left column
 * for y); the basis functions are N_ab(xi, eta) = l_a(xi) l_b(eta), and the
 * element integrals use the (p+1) x (p+1) Gauss rule on the reference square
 * (the integrands are polynomials of degree <= 2p in each variable).
 * Returns -1 for a degenerate element. */
static int qp_element(int p, const double *x, const double *y, double *Ke, double *Me) {
    const int q = p + 1, nv = q * q;
    double xmin = x[0], xmax = x[p], ymin = y[0], ymax = y[p * q];
    double hx = xmax - xmin, hy = ymax - ymin;
    if (!(hx > 0.0) || !(hy > 0.0)) return -1;
    double sx[9], sy[9], gp[9], gw[9], Lx[9], Dx[9], Ly[9], Dy[9];
    for (int a = 0; a <= p; ++a) {
        sx[a] = -1.0 + 2.0 * (x[a] - xmin) / hx;
        sy[a] = -1.0 + 2.0 * (y[a * q] - ymin) / hy;
    }
    gauss_legendre(q, gp, gw);
    memset(Ke, 0, sizeof(double) * nv * nv);
    memset(Me, 0, sizeof(double) * nv * nv);
    const double det = 0.25 * hx * hy;
    for (int i1 = 0; i1 < q; ++i1) {
        lagrange_basis(p, sx, gp[i1], Lx, Dx);
        for (int i2 = 0; i2 < q; ++i2) {
            lagrange_basis(p, sy, gp[i2], Ly, Dy);
            double wq = gw[i1] * gw[i2] * det;
            for (int i = 0; i < nv; ++i) {
                int a = i % q, b = i / q;
                double Ni = Lx[a] * Ly[b];
                double gxi = (2.0 / hx) * Dx[a] * Ly[b], gyi = (2.0 / hy) * Lx[a] * Dy[b];
                for (int j = 0; j < nv; ++j) {
                    int c = j % q, d = j / q;
                    double Nj = Lx[c] * Ly[d];
                    double gxj = (2.0 / hx) * Dx[c] * Ly[d], gyj = (2.0 / hy) * Lx[c] * Dy[d];
                    Ke[i * nv + j] += wq * (gxi * gxj + gyi * gyj);
                    Me[i * nv + j] += wq * Ni * Nj;
                }
            }
        }
    }
    return 0;
}

/* Assemble dense K and M (n_dof x n_dof, column-major, ld = n_dof) over the
 * interior DOFs.  dof_of_node[v] = dof index or -1 for a Dirichlet node.
 * If Kfull/Mfull are non-NULL they receive the matrices over ALL nodes
 * (n_nodes x n_nodes, no elimination) for consistency checks.
 * Returns 0, or -(1+e) for the first element e with non-positive Jacobian. */
int or_assemble(int elem, int64_t n_nodes, const double *xy, int64_t n_elem,
                const int32_t *conn, const int64_t *dof_of_node, int64_t n_dof,
                double *K, double *M, double *Kfull, double *Mfull) {
    memset(K, 0, sizeof(double) * (size_t)n_dof * (size_t)n_dof);
    memset(M, 0, sizeof(double) * (size_t)n_dof * (size_t)n_dof);
    if (Kfull) memset(Kfull, 0, sizeof(double) * (size_t)n_nodes * (size_t)n_nodes);
    if (Mfull) memset(Mfull, 0, sizeof(double) * (size_t)n_nodes * (size_t)n_nodes);
    int nv = elem;
    int p = 0; /* order of a tensor-product element with nv = (p+1)^2 > 4 nodes */
    if (nv > 4) {
        while ((p + 1) * (p + 1) < nv) ++p;
        if ((p + 1) * (p + 1) != nv || p > 8) return -1;
    }
    double *Ke = (double *)malloc(sizeof(double) * 81 * 81);
    double *Me = (double *)malloc(sizeof(double) * 81 * 81);
    for (int64_t e = 0; e < n_elem; ++e) {
        double x[81] = {0}, y[81] = {0};  // the first nv entries are set below
        for (int a = 0; a < nv; ++a) {
            int32_t v = conn[e * nv + a];
            x[a] = xy[2 * (size_t)v];
            y[a] = xy[2 * (size_t)v + 1];
        }
        int rc = (nv == 4) ? q1_element(x, y, Ke, Me) : (nv == 3) ? p1_element(x, y, Ke, Me) : qp_element(p, x, y, Ke, Me);
        if (rc) {
            free(Ke);
            free(Me);
            return (int)(-(1 + e));
        }
        for (int a = 0; a < nv; ++a) {
            int32_t va = conn[e * nv + a];
            for (int b = 0; b < nv; ++b) {
                int32_t vb = conn[e * nv + b];
                if (Kfull) {
                    Kfull[IDX(va, vb, n_nodes)] += Ke[a * nv + b];
                    Mfull[IDX(va, vb, n_nodes)] += Me[a * nv + b];
                }
                int64_t i = dof_of_node[va], j = dof_of_node[vb];
                if (i < 0 || j < 0) continue;
                K[IDX(i, j, n_dof)] += Ke[a * nv + b];
                M[IDX(i, j, n_dof)] += Me[a * nv + b];
            }
        }
    }
    free(Ke);
    free(Me);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Cholesky, standard form, back substitution                                */
/* ------------------------------------------------------------------------ */

/* In-place unblocked Cholesky A = L L^T (lower triangle); the strict upper
 * triangle is zeroed.  Returns 0 or the 1-based index of the first
 * non-positive pivot. */
int or_cholesky(int64_t n, double *A) {
    for (int64_t j = 0; j < n; ++j) {
        double d = A[IDX(j, j, n)];
        for (int64_t k = 0; k < j; ++k) d -= A[IDX(j, k, n)] * A[IDX(j, k, n)];
        if (!(d > 0.0)) return (int)(j + 1);
        d = sqrt(d);
        A[IDX(j, j, n)] = d;
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < n; ++i) {
            double s = A[IDX(i, j, n)];
            for (int64_t k = 0; k < j; ++k) s -= A[IDX(i, k, n)] * A[IDX(j, k, n)];
            A[IDX(i, j, n)] = s / d;
        }
        for (int64_t i = 0; i < j; ++i) A[IDX(i, j, n)] = 0.0;
    }
    return 0;
}

/* C = L^{-1} K L^{-T}: forward-substitute the columns of K (W = L^-1 K),
 * then the columns of W^T (C = L^-1 W^T), then symmetrise. */
void or_standard_form(int64_t n, const double *L, const double *K, double *C) {
    double *W = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t c = 0; c < n; ++c) {
        double *w = W + (size_t)c * n;
        for (int64_t i = 0; i < n; ++i) {
            double s = K[IDX(i, c, n)];
            for (int64_t k = 0; k < i; ++k) s -= L[IDX(i, k, n)] * w[k];
            w[i] = s / L[IDX(i, i, n)];
        }
    }
    /* C(:,c) = L^{-1} (row c of W)^T */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t c = 0; c < n; ++c) {
        double *out = C + (size_t)c * n;
        for (int64_t i = 0; i < n; ++i) {
            double s = W[IDX(c, i, n)];
            for (int64_t k = 0; k < i; ++k) s -= L[IDX(i, k, n)] * out[k];
            out[i] = s / L[IDX(i, i, n)];
        }
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = j + 1; i < n; ++i) {
            double s = 0.5 * (C[IDX(i, j, n)] + C[IDX(j, i, n)]);
            C[IDX(i, j, n)] = s;
            C[IDX(j, i, n)] = s;
        }
    free(W);
}

/* X := L^{-T} X for an n x m block X (back substitution, column by column). */
void or_solve_lt(int64_t n, const double *L, int64_t m, double *X) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t c = 0; c < m; ++c) {
        double *x = X + (size_t)c * n;
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = x[i];
            for (int64_t k = i + 1; k < n; ++k) s -= L[IDX(k, i, n)] * x[k];
            x[i] = s / L[IDX(i, i, n)];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Cyclic two-sided Jacobi, parallel round-robin ordering                    */
/* ------------------------------------------------------------------------ */

/* Diagonalise the symmetric C (n x n, full storage) in place: on return C is
 * diagonal (to the threshold) and Q (n x n) holds the accumulated rotations,
 * C_in = Q diag(C_out) Q^T.  Each step of a sweep pairs every index with one
 * partner (round-robin tournament), so the n/2 rotations of a step act on
 * disjoint index pairs and are applied together.  A pair is rotated when
 * |c_pq| > eps * sqrt(|c_pp c_qq|).  Stops after a sweep without rotations.
 * Returns the number of sweeps, or -1 if max_sweeps were not enough. */
int or_jacobi(int64_t n, double *C, double *Q, int max_sweeps) {
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) Q[IDX(i, j, n)] = (i == j) ? 1.0 : 0.0;
    if (n < 2) return 0;
    int64_t N = (n % 2) ? n + 1 : n; /* odd n: one dummy player */
    int64_t npair = N / 2;
    int64_t *ring = (int64_t *)malloc(sizeof(int64_t) * N);
    int64_t *pp = (int64_t *)malloc(sizeof(int64_t) * npair);
    int64_t *qq = (int64_t *)malloc(sizeof(int64_t) * npair);
    double *cs = (double *)malloc(sizeof(double) * npair);
    double *sn = (double *)malloc(sizeof(double) * npair);
    int64_t *partner = (int64_t *)malloc(sizeof(int64_t) * N);
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * N);
    const double eps = DBL_EPSILON;
    int sweeps = 0;
    for (int64_t i = 0; i < N; ++i) ring[i] = i;
    for (; sweeps < max_sweeps; ++sweeps) {
        int64_t rotations = 0;
        for (int64_t step = 0; step < N - 1; ++step) {
            /* pairs of this step: (ring[k], ring[N-1-k]) */
            for (int64_t k = 0; k < npair; ++k) {
                int64_t a = ring[k], b = ring[N - 1 - k];
                pp[k] = a < b ? a : b;
                qq[k] = a < b ? b : a;
                partner[a] = b;
                partner[b] = a;
                slot[a] = k;
                slot[b] = k;
            }
            /* rotation angles from the current C */
            int64_t rot_step = 0;
#pragma omp parallel for schedule(static) reduction(+ : rot_step)
            for (int64_t k = 0; k < npair; ++k) {
                int64_t p = pp[k], q = qq[k];
                cs[k] = 1.0;
                sn[k] = 0.0;
                if (q >= n) continue;
                double apq = C[IDX(p, q, n)], app = C[IDX(p, p, n)], aqq = C[IDX(q, q, n)];
                if (fabs(apq) <= eps * sqrt(fabs(app * aqq))) continue;
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t);
                cs[k] = c;
                sn[k] = t * c;
                rot_step += 1;
            }
            rotations += rot_step;
            if (rot_step == 0) goto next_step;
            /* new columns p, q of J^T C J: column rotation, then the row
             * rotations of all pairs applied inside the two columns. */
#pragma omp parallel
            {
                double *xp = (double *)malloc(sizeof(double) * n);
                double *xq = (double *)malloc(sizeof(double) * n);
#pragma omp for schedule(static)
                for (int64_t k = 0; k < npair; ++k) {
                    int64_t p = pp[k], q = qq[k];
                    int lone = (q >= n); /* p's partner is the dummy: no column
                                            rotation, but its rows still turn */
                    double c = cs[k], s = sn[k];
                    double *Cp = C + (size_t)p * n, *Cq = lone ? Cp : C + (size_t)q * n;
                    for (int64_t i = 0; i < n; ++i) {
                        xp[i] = c * Cp[i] - s * Cq[i];
                        xq[i] = s * Cp[i] + c * Cq[i];
                    }
                    for (int64_t kk = 0; kk < npair; ++kk) {
                        int64_t r1 = pp[kk], r2 = qq[kk];
                        if (r2 >= n) continue;
                        double c2 = cs[kk], s2 = sn[kk];
                        if (s2 == 0.0) continue;
                        double a1 = xp[r1], a2 = xp[r2];
                        xp[r1] = c2 * a1 - s2 * a2;
                        xp[r2] = s2 * a1 + c2 * a2;
                        a1 = xq[r1];
                        a2 = xq[r2];
                        xq[r1] = c2 * a1 - s2 * a2;
                        xq[r2] = s2 * a1 + c2 * a2;
                    }
                    memcpy(Cp, xp, sizeof(double) * n);
                    if (!lone) memcpy(Cq, xq, sizeof(double) * n);
                }
                free(xp);
                free(xq);
            }
            /* the rotation is built to annihilate c_pq: set it exactly */
#pragma omp parallel for schedule(static)
            for (int64_t k = 0; k < npair; ++k) {
                int64_t p = pp[k], q = qq[k];
                if (q >= n || sn[k] == 0.0) continue;
                C[IDX(p, q, n)] = 0.0;
                C[IDX(q, p, n)] = 0.0;
                double *Qp = Q + (size_t)p * n, *Qq = Q + (size_t)q * n;
                double c = cs[k], s = sn[k];
                for (int64_t i = 0; i < n; ++i) {
                    double a1 = Qp[i], a2 = Qq[i];
                    Qp[i] = c * a1 - s * a2;
                    Qq[i] = s * a1 + c * a2;
                }
            }
        next_step:
            /* rotate the ring: ring[0] fixed, the others move one seat */
            {
                int64_t last = ring[N - 1];
                for (int64_t i = N - 1; i > 1; --i) ring[i] = ring[i - 1];
                ring[1] = last;
            }
        }
        if (rotations == 0) break;
    }
    free(ring);
    free(pp);
    free(qq);
    free(cs);
    free(sn);
    free(partner);
    free(slot);
    return sweeps < max_sweeps ? sweeps + 1 : -1;
}

/* ------------------------------------------------------------------------ */
/* Full generalized eigensolve                                               */
/* ------------------------------------------------------------------------ */

static const double *g_sort_key;
static int cmp_idx(const void *a, const void *b) {
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    double x = g_sort_key[i], y = g_sort_key[j];
    if (x < y) return -1;
    if (x > y) return 1;
    return (i < j) ? -1 : (i > j);
}

/* theta (n) ascending and V (n x n) with V^T M V = I and K V = M V diag(theta).
 * Returns 0, a positive pivot index if M is not positive definite, or -1 if
 * Jacobi did not converge.  *sweeps_out receives the sweep count. */
int or_eigensolve(int64_t n, const double *K, const double *M, double *theta, double *V,
                  int max_sweeps, int *sweeps_out) {
    size_t nn = (size_t)n * (size_t)n;
    double *L = (double *)malloc(sizeof(double) * nn);
    double *C = (double *)malloc(sizeof(double) * nn);
    double *Qm = (double *)malloc(sizeof(double) * nn);
    memcpy(L, M, sizeof(double) * nn);
    int rc = or_cholesky(n, L);
    if (rc) {
        free(L);
        free(C);
        free(Qm);
        return rc;
    }
    or_standard_form(n, L, K, C);
    int sw = or_jacobi(n, C, Qm, max_sweeps);
    if (sweeps_out) *sweeps_out = sw;
    int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * n);
    double *diag = (double *)malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; ++i) {
        perm[i] = i;
        diag[i] = C[IDX(i, i, n)];
    }
    g_sort_key = diag;
    qsort(perm, (size_t)n, sizeof(int64_t), cmp_idx);
    for (int64_t k = 0; k < n; ++k) {
        theta[k] = diag[perm[k]];
        memcpy(V + (size_t)k * n, Qm + (size_t)perm[k] * n, sizeof(double) * n);
    }
    or_solve_lt(n, L, n, V);
    free(perm);
    free(diag);
    free(L);
    free(C);
    free(Qm);
    return sw < 0 ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Spectral application and its adjoint                                      */
/* ------------------------------------------------------------------------ */

/* U(:, j + i*nf) = sum_k theta_k^(-alpha_i/2) (phi_k^T M f_j) phi_k
 * for every forcing j < nf and order i < na.  F is n x nf, U is n x (nf*na). */
void or_apply(int64_t n, const double *theta, const double *V, const double *M,
              int64_t nf, const double *F, int64_t na, const double *alpha, double *U) {
    double *MF = (double *)malloc(sizeof(double) * (size_t)n * nf);
    double *Cf = (double *)malloc(sizeof(double) * (size_t)n * nf);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < nf; ++j)
        for (int64_t r = 0; r < n; ++r) {
            double s = 0.0;
            for (int64_t c = 0; c < n; ++c) s += M[IDX(r, c, n)] * F[IDX(c, j, n)];
            MF[IDX(r, j, n)] = s;
        }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < nf; ++j)
        for (int64_t k = 0; k < n; ++k) {
            double s = 0.0;
            for (int64_t r = 0; r < n; ++r) s += V[IDX(r, k, n)] * MF[IDX(r, j, n)];
            Cf[IDX(k, j, n)] = s;
        }
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t i = 0; i < na; ++i)
        for (int64_t j = 0; j < nf; ++j) {
            double *u = U + (size_t)(j + i * nf) * n;
            for (int64_t r = 0; r < n; ++r) u[r] = 0.0;
            for (int64_t k = 0; k < n; ++k) {
                double w = pow(theta[k], -0.5 * alpha[i]);
                double a = w * Cf[IDX(k, j, n)];
                const double *v = V + (size_t)k * n;
                for (int64_t r = 0; r < n; ++r) u[r] += a * v[r];
            }
        }
    free(MF);
    free(Cf);
}

/* Adjoint of the paired map u_b = sum_k theta_k^(-a_b/2) (phi_k^T M f_b) phi_k
 * for b < nb.  Given GU = dL/du (n x nb): GF = dL/df (n x nb) and
 * galpha = dL/dalpha (nb).  With c = V^T M f, w_k = theta_k^(-a/2),
 * p = V^T GU:  dL/df = M V (w o p),  dL/dalpha = sum_k p_k c_k w_k (-ln theta_k / 2). */
void or_grad(int64_t n, const double *theta, const double *V, const double *M, int64_t nb,
             const double *F, const double *alpha, const double *GU, double *GF, double *galpha) {
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b) {
        double *mf = (double *)malloc(sizeof(double) * n);
        double *c = (double *)malloc(sizeof(double) * n);
        double *p = (double *)malloc(sizeof(double) * n);
        double *y = (double *)malloc(sizeof(double) * n);
        const double *f = F + (size_t)b * n, *gu = GU + (size_t)b * n;
        for (int64_t r = 0; r < n; ++r) {
            double s = 0.0;
            for (int64_t q = 0; q < n; ++q) s += M[IDX(r, q, n)] * f[q];
            mf[r] = s;
        }
        double ga = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            const double *v = V + (size_t)k * n;
            double sc = 0.0, sp = 0.0;
            for (int64_t r = 0; r < n; ++r) {
                sc += v[r] * mf[r];
                sp += v[r] * gu[r];
            }
            c[k] = sc;
            p[k] = sp;
            double w = pow(theta[k], -0.5 * alpha[b]);
            ga += sp * sc * w * (-0.5 * log(theta[k]));
        }
        galpha[b] = ga;
        for (int64_t r = 0; r < n; ++r) y[r] = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            double a = pow(theta[k], -0.5 * alpha[b]) * p[k];
            const double *v = V + (size_t)k * n;
            for (int64_t r = 0; r < n; ++r) y[r] += a * v[r];
        }
        for (int64_t r = 0; r < n; ++r) {
            double s = 0.0;
            for (int64_t q = 0; q < n; ++q) s += M[IDX(r, q, n)] * y[q];
            GF[(size_t)b * n + r] = s;
        }
        free(mf);
        free(c);
        free(p);
        free(y);
    }
}

/* Fractional diffusion (Section "Method", equations model_diffusion and
 * diffusion_solution): with the discrete eigenpairs in place of the
 * continuum ones,
 *   u(t) = sum_k exp(-mu theta_k^(alpha/2) t) (phi_k^T M u0) phi_k.
 * U(:, j + i*nf) = u(t_i; alpha_i, mu_i, u0_j) for j < nf, i < na. */
void or_apply_diffusion(int64_t n, const double *theta, const double *V, const double *M, int64_t nf,
                        const double *U0, int64_t na, const double *alpha, const double *t, const double *mu,
                        double *U) {
    double *MU = (double *)malloc(sizeof(double) * (size_t)n * nf);
    double *Cf = (double *)malloc(sizeof(double) * (size_t)n * nf);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < nf; ++j)
        for (int64_t r = 0; r < n; ++r) {
            double s = 0.0;
            for (int64_t c = 0; c < n; ++c) s += M[IDX(r, c, n)] * U0[IDX(c, j, n)];
            MU[IDX(r, j, n)] = s;
        }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < nf; ++j)
        for (int64_t k = 0; k < n; ++k) {
            double s = 0.0;
            for (int64_t r = 0; r < n; ++r) s += V[IDX(r, k, n)] * MU[IDX(r, j, n)];
            Cf[IDX(k, j, n)] = s;
        }
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t i = 0; i < na; ++i)
        for (int64_t j = 0; j < nf; ++j) {
            double *u = U + (size_t)(j + i * nf) * n;
            for (int64_t r = 0; r < n; ++r) u[r] = 0.0;
            for (int64_t k = 0; k < n; ++k) {
                double w = exp(-mu[i] * pow(theta[k], 0.5 * alpha[i]) * t[i]);
                double a = w * Cf[IDX(k, j, n)];
                const double *v = V + (size_t)k * n;
                for (int64_t r = 0; r < n; ++r) u[r] += a * v[r];
            }
        }
    free(MU);
    free(Cf);
}

/* Adjoint of the paired diffusion map u_b = sum_k w_kb (phi_k^T M u0_b) phi_k,
 * w_kb = exp(-mu_b theta_k^(alpha_b/2) t_b), b < nb.  Given GU = dL/du:
 * with c = V^T M u0, p = V^T GU, e_k = theta_k^(alpha/2):
 *   dL/du0 = M V (w o p)
 *   dL/dalpha = sum_k p_k c_k w_k (-mu t e_k ln(theta_k) / 2)
 *   dL/dt     = sum_k p_k c_k w_k (-mu e_k)
 *   dL/dmu    = sum_k p_k c_k w_k (-t e_k). */
void or_grad_diffusion(int64_t n, const double *theta, const double *V, const double *M, int64_t nb,
                       const double *U0, const double *alpha, const double *t, const double *mu, const double *GU,
                       double *GU0, double *galpha, double *gt, double *gmu) {
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b) {
        double *mu0 = (double *)malloc(sizeof(double) * n);
        double *p = (double *)malloc(sizeof(double) * n);
        double *gy = (double *)malloc(sizeof(double) * n);
        const double *u0 = U0 + (size_t)b * n, *gu = GU + (size_t)b * n;
        for (int64_t r = 0; r < n; ++r) {
            double s = 0.0;
            for (int64_t q = 0; q < n; ++q) s += M[IDX(r, q, n)] * u0[q];
            mu0[r] = s;
        }
        double ga = 0.0, g_t = 0.0, g_mu = 0.0;
        for (int64_t r = 0; r < n; ++r) gy[r] = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            const double *v = V + (size_t)k * n;
            double sc = 0.0, sp = 0.0;
            for (int64_t r = 0; r < n; ++r) {
                sc += v[r] * mu0[r];
                sp += v[r] * gu[r];
            }
            p[k] = sp;
            double e = pow(theta[k], 0.5 * alpha[b]);
            double w = exp(-mu[b] * e * t[b]);
            double q = sp * sc * w;
            ga += q * (-mu[b] * t[b] * e * 0.5 * log(theta[k]));
            g_t += q * (-mu[b] * e);
            g_mu += q * (-t[b] * e);
            for (int64_t r = 0; r < n; ++r) gy[r] += w * sp * v[r];
        }
        galpha[b] = ga;
        gt[b] = g_t;
        gmu[b] = g_mu;
        for (int64_t r = 0; r < n; ++r) {
            double s = 0.0;
            for (int64_t q = 0; q < n; ++q) s += M[IDX(r, q, n)] * gy[q];
            GU0[(size_t)b * n + r] = s;
        }
        free(mu0);
        free(p);
        free(gy);
    }
}

/* Number of negative pivots of the LDL^T factorisation (no pivoting) of the
 * symmetric A (n x n, destroyed).  By Sylvester's law of inertia this counts
 * the eigenvalues of the pencil below sigma when A = K - sigma M (Section
 * "Eigenvalue counting").  Returns -1 on a zero pivot. */
int64_t or_inertia_negative(int64_t n, double *A) {
    int64_t neg = 0;
    for (int64_t j = 0; j < n; ++j) {
        double d = A[IDX(j, j, n)];
        if (d == 0.0) return -1;
        if (d < 0.0) ++neg;
#pragma omp parallel for schedule(static)
        for (int64_t c = j + 1; c < n; ++c) {
            double l = A[IDX(j, c, n)] / d;
            if (l == 0.0) continue;
            for (int64_t r = j + 1; r < n; ++r) A[IDX(r, c, n)] -= l * A[IDX(r, j, n)];
        }
    }
    return neg;
}

/* The same count for a symmetric band matrix: AB holds the lower band,
 * AB[(r - c) + c * (bw + 1)] = A(r, c) for 0 <= r - c <= bw (destroyed).
 * LDL^T without pivoting keeps the band, so the cost is about n bw^2 / 2.
 * Returns -1 on a zero pivot. */
int64_t or_inertia_negative_band(int64_t n, int64_t bw, double *AB) {
    const int64_t ld = bw + 1;
    int64_t neg = 0;
    for (int64_t j = 0; j < n; ++j) {
        double d = AB[(size_t)j * ld];
        if (d == 0.0) return -1;
        if (d < 0.0) ++neg;
        int64_t last = j + bw < n - 1 ? j + bw : n - 1;
        for (int64_t c = j + 1; c <= last; ++c) {
            double l = AB[(size_t)(c - j) + (size_t)j * ld] / d;
            if (l == 0.0) continue;
            for (int64_t r = c; r <= last; ++r)
                AB[(size_t)(r - c) + (size_t)c * ld] -= l * AB[(size_t)(r - j) + (size_t)j * ld];
        }
    }
    return neg;
}
