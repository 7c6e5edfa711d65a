/*
 * fraclap -- MI355X (gfx950) library for the spectral fractional Poisson
 * problem by eigenfunction expansion (Carlson, Kirby, Sundar, "A Scalable
 * Framework for Solving Fractional Diffusion Equations").
 *
 * The method (Section "Method"): with the Galerkin pencil
 *     K_ij = <grad e_i, grad e_j>,   M_ij = <e_i, e_j>      (eq. discrete_laplace)
 * compute ALL n generalized eigenpairs K phi_k = theta_k M phi_k with
 * phi_j^T M phi_k = delta_jk (orthonormality: Section "Post-processing"), then
 * for any forcing f and fractional order alpha
 *     v = sum_k theta_k^(-alpha/2) <f, phi_k> phi_k,   <f, phi_k> = phi_k^T M f
 * (the equations for g and v in Section "Method"; the basis is computed once
 * and reused for every forcing, same section).
 *
 * Conventions
 *  - Dense matrices are column-major; element (i, j) of an array with leading
 *    dimension ld is at X[i + j*ld].  All floating point is IEEE double unless
 *    a function says otherwise.
 *  - "device" pointers are HIP device memory (e.g. the data pointer of a torch
 *    tensor on cuda:N); "host" pointers are ordinary process memory.  Device
 *    pointers are borrowed for the duration of the stream-ordered work; host
 *    inputs are copied before the call returns.  Output buffers are always
 *    allocated by the caller.  The library owns K, M, theta, V and its
 *    workspace until fl_op_destroy.
 *  - Every call returns FL_OK (0) or a negative status; the message of the
 *    last failure is available from fl_last_error.  Argument validation runs
 *    before any device work, so a rejected call leaves all buffers untouched.
 *  - Synchrony: fl_assemble, fl_op_from_dense, fl_eigensolve and the fl_d*
 *    stage calls return after their device work has completed;
 *    fl_apply_fractional, fl_apply_diffusion, fl_apply_graph and the adjoints
 *    (unless they return per-column derivatives to the host) are
 *    asynchronous on the context stream.
 *  - Streams: work is queued on the context's current stream
 *    (fl_ctx_set_stream).  Each operator keeps one application workspace per
 *    stream, and products split along k use a buffer owned by their stream,
 *    so applications queued on different streams never share intermediate
 *    buffers.  Calls on one stream are ordered by that stream.
 *  - Threading: one context per host thread.
 */
#ifndef FRACLAP_H
#define FRACLAP_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fl_ctx fl_ctx; /* device, borrowed stream, last error */
typedef struct fl_op fl_op;   /* one discretised domain: K, M; after eigensolve theta, V */

enum {
    FL_OK = 0,
    FL_EINVAL = -1,   /* bad argument (sizes, NaN/Inf input, bad mesh, alpha with theta_1 <= 0) */
    FL_ENOMEM = -2,   /* device allocation failed */
    FL_EHIP = -3,     /* HIP runtime error */
    FL_ENOTSPD = -4,  /* M (or a matrix to factor) is not positive definite; info->index = pivot */
    FL_ENOCONV = -5,  /* an iterative stage did not converge; info->index = stage */
    FL_ESTATE = -6,   /* call out of order (apply before eigensolve) */
    FL_EIO = -7       /* a file could not be read or written, or failed its checks */
};
enum { FL_ELEM_P1 = 3, FL_ELEM_Q1 = 4 };
#define FL_ELEM_QP(p) (((p) + 1) * ((p) + 1))
enum { FL_FP64 = 0, FL_MIXED = 1 };

/* Eigensolve stages, in order (indices into fl_eig_info.stage_ms). */
enum {
    FL_STAGE_POTRF = 0, /* M = L L^T */
    FL_STAGE_SYGST = 1, /* C = L^-1 K L^-T */
    FL_STAGE_SY2SB = 2, /* C -> symmetric band (Householder panels, MFMA updates) */
    FL_STAGE_SB2ST = 3, /* band -> tridiagonal (bulge chasing) */
    FL_STAGE_STEDC = 4, /* tridiagonal divide and conquer */
    FL_STAGE_Q2 = 5,    /* back-transform by the bulge-chasing reflectors */
    FL_STAGE_Q1 = 6,    /* back-transform by the band-reduction reflectors */
    FL_STAGE_TRSM = 7,  /* V = L^-T Z */
    FL_STAGE_REFINE = 8,/* mixed mode: eigenpair refinement */
    FL_NSTAGES = 9
};

typedef struct fl_eig_opts {
    int32_t band;             /* band width of the two-stage reduction (0 = default 64) */
    int32_t leaf;             /* divide-and-conquer leaf size (0 = default 32) */
    int32_t refine_max_iters; /* refinement steps (-1 = default: 0 in FP64 mode; in mixed mode 2,
                                 or 3 with FL_MIXED_FP32_BAND) */
    double refine_tol;        /* stop refining when max |(I - V^T M V)_ij| is below this
                                 (0 = default 1e-13) */
    int32_t mixed_flags;      /* mixed mode: 0 = FP64 band reduction, FP32 back-transforms;
                                 FL_MIXED_FP32_BAND = the band reduction in FP32 as well (its
                                 rounding is amplified by 1/gap in the eigenvectors, so more
                                 refinement steps are needed) */
} fl_eig_opts;

enum { FL_MIXED_FP32_BAND = 1 };

typedef struct fl_eig_info {
    int32_t status;           /* FL_OK or the failing status */
    int64_t index;            /* FL_ENOTSPD: 1-based pivot; FL_ENOCONV: stage */
    int32_t refine_iters;     /* mixed mode: sweeps done */
    double refine_resid;      /* mixed mode: last max |I - X^T M X| entry */
    double stage_ms[FL_NSTAGES]; /* per-stage device time (HIP events) */
    double total_ms;
    double flops_nominal;     /* 9 n^3 */
} fl_eig_info;

/* ---- context ------------------------------------------------------------ */
/* device: HIP ordinal.  hip_stream: a hipStream_t to borrow (NULL = the
 * legacy default stream).  *out receives the context. */
int fl_ctx_create(int device, void *hip_stream, fl_ctx **out);
int fl_ctx_set_stream(fl_ctx *ctx, void *hip_stream);
/* Frees the context.  The uncached buffer that an eigensolve of this context
 * allocated for the bulge chase's band ((2 band + 1) n doubles for the
 * largest n solved) is not freed: uncached device memory stays allocated until
 * the process ends. */
void fl_ctx_destroy(fl_ctx *ctx);
/* Message for the last non-OK status on this context ("" if none). */
const char *fl_last_error(const fl_ctx *ctx);

/* ---- input stage: the discretised pencil (eq. discrete_laplace) ----------
 * Assemble K and M for a mesh with homogeneous Dirichlet data (Section
 * "Accuracy"): Dirichlet nodes are eliminated, interior nodes become DOFs in
 * node order.  elem = FL_ELEM_Q1 (4 nodes, counter-clockwise, axis-aligned
 * rectangles), FL_ELEM_P1 (3 nodes, counter-clockwise), or FL_ELEM_QP(p) =
 * (p+1)^2 for tensor-product Lagrange elements of order 2 <= p <= 8 on
 * axis-aligned rectangles (the order sweep of Section "Accuracy"): nodes in
 * lexicographic order a + (p+1) b, node (a, b) at (x of (a, 0), y of (0, b)),
 * x and y increasing.  Exact element integrals (consistent mass).  xy: host, n_nodes x 2 row-major (x, y);
 * conn: host, n_elem x elem row-major; dirichlet: host, n_nodes flags.
 * *n_dof receives n; dof_of_node (host, n_nodes, may be NULL) receives the
 * DOF index of each node or -1.  FL_EINVAL for NaN/Inf coordinates, node
 * indices out of range, clockwise or degenerate elements, non-rectangular Q1
 * elements, order-p elements whose nodes are not an increasing tensor
 * lattice, or no interior node. */
int fl_assemble(fl_ctx *ctx, int elem, int64_t n_nodes, const double *xy, int64_t n_elem,
                const int32_t *conn, const uint8_t *dirichlet, fl_op **out, int64_t *n_dof,
                int64_t *dof_of_node);
/* Same mesh input, for pencils too large for dense storage: the element
 * contributions go straight into the values of the CSR pattern (bitwise the
 * CSR copies fl_assemble makes), and no dense K or M is kept.  Such an
 * operator serves fl_inertia_count, fl_eigensolve_interval, fl_op_save and,
 * once eigenpairs are installed, the applications; fl_eigensolve,
 * fl_eigensolve_batched and fl_op_matrices refuse it with FL_ESTATE. */
int fl_assemble_sparse(fl_ctx *ctx, int elem, int64_t n_nodes, const double *xy, int64_t n_elem,
                       const int32_t *conn, const uint8_t *dirichlet, fl_op **out, int64_t *n_dof,
                       int64_t *dof_of_node);
/* Wrap an existing symmetric pencil.  K, M: n x n, leading dimension ld,
 * host (on_device = 0) or device (1).  FL_EINVAL for NaN/Inf entries. */
int fl_op_from_dense(fl_ctx *ctx, int64_t n, const double *K, const double *M, int64_t ld, int on_device,
                     fl_op **out);
int64_t fl_op_n(const fl_op *op);
/* Copy K and/or M (either may be NULL) out to host or device memory. */
int fl_op_matrices(const fl_op *op, double *K, double *M, int64_t ld, int on_device);
void fl_op_destroy(fl_op *op);

/* ---- the eigensolve ------------------------------------------------------
 * All n pairs of K phi = theta M phi, theta ascending, V^T M V = I
 * (eq. discrete_laplace, Section "Post-processing").  Stages: FL_STAGE_*.
 * precision = FL_FP64 runs every stage in FP64; FL_MIXED runs both
 * back-transforms (and, with FL_MIXED_FP32_BAND, the band reduction) in FP32
 * on the matrix cores and restores FP64 accuracy by eigenpair refinement.
 * opts/info may be NULL.  Synchronous.
 * FL_ENOTSPD if M is not positive definite (info->index = pivot). */
int fl_eigensolve(fl_op *op, int precision, const fl_eig_opts *opts, fl_eig_info *info);
/* Many independent problems (one per domain; the basis of each is computed
 * once and reused for every forcing, Section "Method") in one persistent
 * launch: each workgroup takes the next problem, largest n first, from an
 * atomic counter and runs Cholesky, reduction to standard form, Householder
 * tridiagonalisation, tridiagonal divide and conquer (implicit-QL leaves,
 * secular-equation merges) and the back-transforms on its own, in FP64.
 * ops: host array of count distinct operators of this context's device, each
 * with 1 <= n <= 1024.  precision must be FL_FP64.  On return each op holds
 * theta ascending and M-orthonormal V, as after fl_eigensolve.  infos (host,
 * count entries, may be NULL) receive per-problem status and index
 * (FL_ENOTSPD: 1-based pivot; FL_ENOCONV: index 1, the tridiagonal divide
 * and conquer did not converge) and, in total_ms, the time of the whole
 * launch.  Returns FL_OK, or the status of the first failed
 * problem (the others are still solved).  Workspace: about 4 n^2 doubles per
 * problem, allocated and released by the call.  Synchronous. */
int fl_eigensolve_batched(fl_ctx *ctx, int64_t count, fl_op *const *ops, int precision, fl_eig_info *infos);
/* The same solve in two halves, so that the caller can queue other work
 * (on other streams) while the launch runs: fl_eigensolve_batched_begin
 * checks the arguments as above, allocates the workspace and queues the
 * launch on the context's stream, then returns; *out (host) receives the
 * handle of the launch in flight, or NULL when count == 0.  The operators
 * must not be used or destroyed until fl_eigensolve_batched_wait(handle,
 * infos) has returned: it waits for the launch, fills infos (as above; may
 * be NULL), releases the workspace and the handle (in every case, errors
 * included) and returns the status fl_eigensolve_batched would return.
 * The synchronous call is begin followed by wait. */
typedef struct fl_batch fl_batch;
int fl_eigensolve_batched_begin(fl_ctx *ctx, int64_t count, fl_op *const *ops, int precision, fl_batch **out);
int fl_eigensolve_batched_wait(fl_batch *batch, fl_eig_info *infos);
/* Copy theta (n) and V (n x n, ld ldv; V may be NULL) out. */
int fl_eigenpairs(const fl_op *op, double *theta, double *V, int64_t ldv, int on_device);
/* Install eigenpairs computed elsewhere (resume, or testing the apply path
 * alone).  theta must be positive. */
int fl_op_set_eigenpairs(fl_op *op, const double *theta, const double *V, int64_t ldv, int on_device);

/* ---- persistence: the basis is computed once and reused for every later
 * forcing (Section "Method", the paragraph after the equation for v) --------
 * fl_op_save writes the pencil (its CSR pattern and the K and M values, and
 * whether the operator keeps a dense copy), and
 * theta, V and how they were obtained (precision, refinement steps, last
 * refinement residual) when present, with a SHA-256 of the pencil and one of
 * the whole file; the file is written under path + ".part" and renamed when
 * complete.  fl_op_load reads such a file into a new operator of ctx's device
 * (dense K and M rebuilt from the pattern unless the saved operator had
 * none), after checking the magic, the
 * version, the sizes, the pattern's indices and the file checksum: FL_EIO on
 * any failure (nothing is created).  Both synchronous. */
int fl_op_save(const fl_op *op, const char *path);
int fl_op_load(fl_ctx *ctx, const char *path, fl_op **out);
/* n, whether eigenpairs are present, and how they were obtained (precision
 * FL_FP64, FL_MIXED, or -1 when installed by fl_op_set_eigenpairs); any
 * output may be NULL. */
int fl_op_info(const fl_op *op, int64_t *n, int *has_eig, int *precision, int *refine_iters, double *refine_resid);

/* ---- eigenvalue counting (Section "Eigenvalue counting") ------------------
 * By Sylvester's law of inertia the number of eigenvalues of
 * K phi = theta M phi below sigma equals the number of negative pivots of an
 * LDL^T factorisation of K - sigma M.  The pencil's pattern is renumbered to
 * a small bandwidth (natural or reverse Cuthill-McKee numbering, whichever is
 * narrower; a symmetric permutation keeps the inertia; computed once per
 * operator on the host), and the banded matrix of each shift is factored
 * without pivoting on the device, one workgroup per shift.
 * sigma: host, nshift shifts; counts: host, nshift results (-1 where a pivot
 * was exactly zero); bandwidth (host, may be NULL) receives the bandwidth
 * used.  FL_EINVAL for a non-finite shift, an operator without a sparse
 * pattern, or a bandwidth above 511.  Needs no eigenpairs.  Synchronous. */
int fl_inertia_count(fl_op *op, int64_t nshift, const double *sigma, int64_t *counts, int64_t *bandwidth);

/* ---- spectrum slicing (Sections "Solving for all eigenpairs in an
 * interval", "Partitioning" (greedy partitioning) and "Post-processing") ---
 * All eigenpairs with lo <= theta < hi, for pencils of any size held in
 * sparse form (see fl_assemble_sparse): the interval's count from inertia
 * counts; greedy partitioning into slices of at most max_per_slice
 * (<= 500) eigenvalues (7 rounds of batched counts below every split
 * point, splits moved to equal shares of the piecewise-linear cumulative
 * count, the best partition kept, overloaded slices halved); per slice one
 * banded LDL^T of K - sigma_s M at its midpoint and shift-invert subspace
 * iteration with 2 m_s + 16 vectors and Rayleigh-Ritz on the batched
 * eigensolver, all slices together, until each slice holds exactly its m_s
 * Ritz pairs with relative residuals ||K x - theta M x|| / (max(theta, b_s)
 * ||M x||) below tol (b_s: the slice's upper end; the m_s eigenvalues inside
 * are known from the counts), then one Newton-Schulz step V := V (3 I -
 * V^T M V) / 2 over all returned vectors.  theta (device, cap) receives the eigenvalues ascending and V
 * (device, n x cap, ld ldv) M-orthonormal eigenvectors.  info (may be NULL)
 * receives the count (also when it exceeds cap: then FL_EINVAL), the number
 * of slices, the largest slice load, partitioning rounds, iterations and the
 * largest residual.  FL_ENOCONV if the iteration did not converge within
 * 200 steps.  Synchronous. */
typedef struct fl_slice_info {
    int64_t count, slices, max_load, partition_rounds, iterations;
    double max_residual;
} fl_slice_info;
int fl_eigensolve_interval(fl_op *op, double lo, double hi, int64_t max_per_slice, double tol, int64_t cap,
                           double *theta, double *V, int64_t ldv, fl_slice_info *info);

/* ---- spectral application (the equation for v, Section "Method") ---------
 * F: device, n x nf (ld ldf).  alpha: host, na orders in [0, 2].
 * paired = 0: U (device, n x nf*na, ld ldu) column j + i*nf = v(alpha_i, f_j).
 * paired = 1: requires na == nf; column b = v(alpha_b, f_b).
 * Computes G = M F, C = V^T G, W_ki = theta_k^(-alpha_i/2) (alpha = 0 gives
 * exactly 1), U = V (W o C) with the scaling fused into the GEMM's operand
 * staging.  FL_ESTATE before an eigensolve; FL_EINVAL for alpha outside
 * [0, 2] or non-finite. */
int fl_apply_fractional(fl_op *op, int64_t nf, const double *F, int64_t ldf, int64_t na, const double *alpha,
                        int paired, double *U, int64_t ldu);
/* Adjoint of the paired map (f_b, alpha_b) -> u_b, b < nb.  GU = dL/du
 * (device n x nb).  With c = V^T M f, w = theta^(-alpha/2), p = V^T GU:
 *   GF = dL/df = M V (w o p)            (device n x nb, ld ldgf; may be NULL)
 *   galpha_b = dL/dalpha_b = sum_k p_k c_k w_k (-ln(theta_k)/2)
 *                                      (galpha: host nb; may be NULL).
 * Synchronises the stream when galpha is requested. */
int fl_grad_apply(fl_op *op, int64_t nb, const double *F, int64_t ldf, const double *alpha, const double *GU,
                  int64_t ldgu, double *GF, int64_t ldgf, double *galpha);

/* Same result as fl_apply_fractional (bit for bit), from a graph: the first
 * call with a given set of arguments (operator, sizes, the F and U pointers
 * and leading dimensions, and the values of alpha) captures the sequence
 * G = M F, C = V^T G, weights, scaled product into a HIP graph with its own
 * workspace; every later call with the same arguments replays it.  Replays
 * run on a stream owned by the context, ordered after the work already
 * queued on the context stream and before the work queued after the call.
 * F is read and U written at replay time, so a caller may refill F between
 * calls.  Up to 8 graphs are kept per operator (least recently replayed
 * evicted); they are released with the operator.  FL_ESTATE if the context
 * stream is itself being captured.  Asynchronous. */
int fl_apply_graph(fl_op *op, int64_t nf, const double *F, int64_t ldf, int64_t na, const double *alpha,
                   int paired, double *U, int64_t ldu);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): the same result as
 * fl_apply_fractional, with every intermediate (G, C, W and the split-k
 * partial sums of V^T G) in one fixed device array of the library of
 * FL_NOALLOC_SCRATCH_BYTES per device, held until the process ends.  Nothing
 * is allocated and nothing synchronises.  FL_EINVAL when (2 nf + na) n
 * doubles exceed the array (checked before any device work).  All calls on
 * one device share its array: calls that overlap on a device (different
 * streams or threads) race; calls on one stream are ordered.  Asynchronous. */
#define FL_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int fl_apply_fractional_noalloc(fl_op *op, int64_t nf, const double *F, int64_t ldf, int64_t na, const double *alpha,
                                int paired, double *U, int64_t ldu);

/* ---- fractional diffusion (Section "Method", equations model_diffusion and
 * diffusion_solution; the exact solution of Section "Accuracy", equations
 * diffusion_ics and diffusion_sols) ------------------------------------------
 * u(t) = sum_k exp(-mu theta_k^(alpha/2) t) <u0, phi_k> phi_k,
 * <u0, phi_k> = phi_k^T M u0.  U0: device n x nf (ld ldu0).  alpha, t, mu:
 * host, na values each (alpha in [0, 2], t >= 0, mu >= 0, finite).
 * paired = 0: U (device n x nf*na, ld ldu) column j + i*nf = u(t_i; alpha_i,
 * mu_i, u0_j); paired = 1: requires na == nf, column b uses parameter set b.
 * Same pipeline as fl_apply_fractional with W_ki = exp(-mu_i t_i
 * theta_k^(alpha_i/2)) (t = 0 gives exactly 1).  Asynchronous. */
int fl_apply_diffusion(fl_op *op, int64_t nf, const double *U0, int64_t ldu0, int64_t na, const double *alpha,
                       const double *t, const double *mu, int paired, double *U, int64_t ldu);
/* Adjoint of the paired diffusion map, b < nb.  GU = dL/du (device n x nb).
 * With c = V^T M u0, w = exp(-s theta^(alpha/2)), s = mu t, p = V^T GU:
 *   GU0 = dL/du0 = M V (w o p)                     (device; may be NULL)
 *   galpha_b = sum_k p_k c_k w_k (-s theta_k^(alpha/2) ln(theta_k) / 2)
 *   gt_b = mu_b sum_k p_k c_k w_k (-theta_k^(alpha/2)),  gmu_b = t_b (same sum)
 * (host, nb each; each may be NULL).  Synchronises the stream when any of
 * them is requested. */
int fl_grad_diffusion(fl_op *op, int64_t nb, const double *U0, int64_t ldu0, const double *alpha, const double *t,
                      const double *mu, const double *GU, int64_t ldgu, double *GU0, int64_t ldgu0, double *galpha,
                      double *gt, double *gmu);

/* ---- stage entry points (device pointers; synchronous) -------------------
 * Exposed so that each stage can be checked on its own. */
/* C = alpha op(A) op(B) + beta C, FP64 on the matrix cores.  ta/tb: 0 = N, 1 = T. */
int fl_dgemm(fl_ctx *ctx, int ta, int tb, int64_t m, int64_t n, int64_t k, double alpha, const double *A,
             int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc);
/* In-place Cholesky A = L L^T of the lower triangle; the strict upper
 * triangle is left undefined.  *info = 0 or the 1-based failing pivot. */
int fl_dpotrf(fl_ctx *ctx, int64_t n, double *A, int64_t lda, int64_t *info);
/* K := L^-1 K L^-T (full symmetric storage in and out); L lower from fl_dpotrf. */
int fl_dsygst(fl_ctx *ctx, int64_t n, const double *L, int64_t ldl, double *K, int64_t ldk);
/* All eigenpairs of the symmetric tridiagonal (d: n diagonal, e: n-1
 * off-diagonal; both device, overwritten): d := eigenvalues ascending,
 * Z (n x n, ld ldz) := orthonormal eigenvectors.  Divide and conquer. */
int fl_dstedc(fl_ctx *ctx, int64_t n, double *d, double *e, double *Z, int64_t ldz);
/* Two-stage tridiagonalisation of the symmetric A (full storage, destroyed):
 * d (n), e (n-1) receive T; if Q is non-NULL it receives the orthogonal
 * n x n Q with A = Q T Q^T. */
int fl_dsytrd_2stage(fl_ctx *ctx, int64_t n, double *A, int64_t lda, int band, double *d, double *e, double *Q,
                     int64_t ldq);
/* All eigenpairs of the symmetric A (full storage, destroyed): w ascending,
 * Z orthonormal (n x n, ld ldz). */
int fl_dsyevd(fl_ctx *ctx, int64_t n, double *A, int64_t lda, int band, double *w, double *Z, int64_t ldz);

/* ---- launch-shape autotuner ------------------------------------------------
 * The matrix-core products consult a process-wide table that maps a product
 * shape to a launch shape.  kind: FL_TUNE_F64 / FL_TUNE_F32 (C = op(A) op(B),
 * m x n x k) or FL_TUNE_SCALED (the fused spectral-application product,
 * n x ncols x n; ta = tb = 0).  variant: FL_GV_SQUARE16 / FL_GV_SQUARE32
 * (128 x 128 tiles, k-step 16 / 32), FL_GV_THIN (256 x 64 tiles, n <= 64);
 * split: k split factor (plain products); group: row tiles per band of the
 * XCD-grouped tile order (spectral product).  Shapes match on kind, ta, tb,
 * m, n and the power-of-two bucket of k.  fl_gemm_tune times every candidate
 * on ctx's stream on synthetic operands (median of reps after one warm-up),
 * records the fastest and returns it (ms = its time).  fl_gemm_tuning_set
 * installs an entry (e.g. one saved by an earlier process; FL_EINVAL if
 * malformed); fl_gemm_tuning_count / fl_gemm_tuning_get enumerate the table. */
enum { FL_TUNE_F64 = 0, FL_TUNE_F32 = 1, FL_TUNE_SCALED = 2 };
enum { FL_GV_AUTO = 0, FL_GV_SQUARE16 = 1, FL_GV_SQUARE32 = 2, FL_GV_THIN = 3 };
typedef struct fl_gemm_choice {
    int32_t kind, ta, tb;
    int64_t m, n, k;
    int32_t variant, split, group;
    double ms;
} fl_gemm_choice;
int fl_gemm_tune(fl_ctx *ctx, int kind, int ta, int tb, int64_t m, int64_t n, int64_t k, int reps,
                 fl_gemm_choice *best);
int fl_gemm_tuning_set(const fl_gemm_choice *choice);
int64_t fl_gemm_tuning_count(void);
int fl_gemm_tuning_get(int64_t index, fl_gemm_choice *out);
void fl_gemm_tuning_clear(void);

/* ---- diagnostics ----------------------------------------------------------
 * Per-kernel timing for the library's main kernels ("q2_apply", "sb2st",
 * "scaled_gemm", "batched_eig"): while enabled, HIP events are recorded on
 * the launching stream around each launch (not inside a graph capture).
 * fl_kernel_time waits for the recorded events, returns the launch count and
 * the summed duration for `name`, and clears them; disabling the timer
 * releases every event not yet collected.  Process-wide; FL_EINVAL for NULL
 * arguments. */
int fl_kernel_timing(int enable);
int fl_kernel_time(const char *name, int64_t *count, double *total_ms);
/* Measured ceilings of ctx's device (best of 5 timed runs after one
 * warm-up): FP64 and FP32 matrix-core rates in TFLOP/s (independent
 * 16x16x4 MFMA chains in every wave, two waves per SIMD) and the HBM rate of
 * a plain copy of copy_bytes in GB/s (bytes read plus bytes written).  Any
 * output may be NULL.  FL_EINVAL for a copy under 1 MiB.  Synchronous. */
int fl_measure_peaks(fl_ctx *ctx, double *fp64_tflops, double *fp32_tflops, double *copy_gbs, int64_t copy_bytes);

#ifdef __cplusplus
}
#endif
#endif /* FRACLAP_H */
