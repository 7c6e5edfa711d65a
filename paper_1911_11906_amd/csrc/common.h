// Shared declarations of the fraclap HIP library (gfx950 / MI355X).
// All dense matrices are column-major, element (i, j) at A[i + j * lda].
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include "../../include/fraclap.h"

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

#define FL_DIV_UP(a, b) (((a) + (b) - 1) / (b))

// One GEMM problem C = alpha * op(A) op(B) + beta * C, op(A) m x k, op(B) k x n.
struct GemmProblem {
    int64_t m, n, k;
    const double* A;
    int64_t lda;
    const double* B;
    int64_t ldb;
    double* C;
    int64_t ldc;
    double alpha, beta;
};

// Caller-provided workspace for the partial sums of a split-k product
// (bytes == 0: never split).  Without one, a product uses a buffer owned by
// its stream.
struct SplitWs {
    void* p;
    size_t bytes;
};

// The split-k buffer owned by stream s on the current device (allocated on
// first use, never while s is being captured; {null, 0} if unavailable).
SplitWs fl_stream_splitk_ws(hipStream_t s);

// Tuned launch shapes (tune.hip): product kind (FL_TUNE_*), variant
// (FL_GV_*) and split factor; the enums are part of the public header.
struct GemmChoice {
    int variant = FL_GV_AUTO;  // FL_GV_AUTO: built-in heuristics
    int split = 1;             // split-k factor (plain products)
    int group = 8;             // row tiles per band of the XCD-grouped order (spectral product)
};
// Tuned choice for a product shape (k compared by its power-of-two bucket);
// FL_GV_AUTO when none was recorded.
GemmChoice tuned_choice(int kind, int ta, int tb, int64_t m, int64_t n, int64_t k);
// One product with an explicit choice, alpha = 1, beta = 0 (for the tuner).
hipError_t fl_gemm_choice_launch(hipStream_t s, int kind, int ta, int tb, int64_t m, int64_t n, int64_t k,
                                 const void* A, int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc,
                                 const GemmChoice& c);

// Launchers (stream-ordered, asynchronous).  ta / tb: 0 = N, 1 = T.
// lower != 0 skips output tiles strictly above the diagonal (SYRK-style
// updates of a lower-stored symmetric matrix; diagonal tiles are written in
// full).
hipError_t fl_dgemm(hipStream_t s, int ta, int tb, int64_t m, int64_t n, int64_t k, double alpha,
                    const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                    int64_t ldc, int lower = 0);
// Same, with the split-k workspace given by the caller (nothing allocated).
hipError_t fl_dgemm_ws(hipStream_t s, int ta, int tb, int64_t m, int64_t n, int64_t k, double alpha,
                       const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                       int64_t ldc, const SplitWs* ws);
// GEMM with one triangular operand whose zero part is skipped tile by tile:
// kt = FL_KT_A_LOWER (op(A)[i][k] = 0 for k > i), FL_KT_A_UPPER (for k < i),
// FL_KT_B_LOWER (op(B)[k][j] = 0 for k < j), FL_KT_NONE (plain).  The zero
// part must hold zeros (only whole tiles are skipped).  No split-K.
enum { FL_KT_NONE = 0, FL_KT_A_LOWER = 1, FL_KT_A_UPPER = 2, FL_KT_B_LOWER = 3 };
hipError_t fl_dgemm_tri(hipStream_t s, int ta, int tb, int64_t m, int64_t n, int64_t k, double alpha,
                        const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                        int64_t ldc, int lower, int kt);
// Batched GEMM over problems held in DEVICE memory; grid sized for the largest
// (max_m, max_n) and each tile exits early if outside its own problem.
hipError_t fl_dgemm_batched(hipStream_t s, int ta, int tb, const GemmProblem* dev_probs, int count,
                            int64_t max_m, int64_t max_n);

// FP32 GEMM (mixed-precision mode): same conventions.
hipError_t fl_sgemm(hipStream_t s, int ta, int tb, int64_t m, int64_t n, int64_t k, float alpha,
                    const float* A, int64_t lda, const float* B, int64_t ldb, float beta, float* C,
                    int64_t ldc, int lower = 0);

hipError_t fl_d2s(hipStream_t s, int64_t m, int64_t n, const double* A, int64_t lda, float* B, int64_t ldb);
hipError_t fl_s2d(hipStream_t s, int64_t m, int64_t n, const float* A, int64_t lda, double* B, int64_t ldb);

// type-dispatched GEMM (FP64 or FP32 matrix cores)
inline hipError_t fl_gemm_t(hipStream_t s, int ta, int tb, int64_t m, int64_t n, int64_t k, double alpha,
                            const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                            int64_t ldc, int lower = 0) {
    return fl_dgemm(s, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, lower);
}
inline hipError_t fl_gemm_t(hipStream_t s, int ta, int tb, int64_t m, int64_t n, int64_t k, double alpha,
                            const float* A, int64_t lda, const float* B, int64_t ldb, double beta, float* C,
                            int64_t ldc, int lower = 0) {
    return fl_sgemm(s, ta, tb, m, n, k, (float)alpha, A, lda, B, ldb, (float)beta, C, ldc, lower);
}

// small helpers
hipError_t fl_copy_matrix(hipStream_t s, int64_t m, int64_t n, const double* A, int64_t lda, double* B,
                          int64_t ldb);
hipError_t fl_transpose(hipStream_t s, int64_t m, int64_t n, const double* A, int64_t lda, double* B,
                        int64_t ldb);
hipError_t fl_fill(hipStream_t s, int64_t m, int64_t n, double v, double* A, int64_t lda);
// upper triangle of the n x n A := transpose of its strict lower triangle
hipError_t fl_mirror_lower(hipStream_t s, int64_t n, double* A, int64_t lda);
hipError_t fl_mirror_lower_f(hipStream_t s, int64_t n, float* A, int64_t lda);
inline hipError_t fl_mirror_lower_t(hipStream_t s, int64_t n, double* A, int64_t lda) {
    return fl_mirror_lower(s, n, A, lda);
}
inline hipError_t fl_mirror_lower_t(hipStream_t s, int64_t n, float* A, int64_t lda) {
    return fl_mirror_lower_f(s, n, A, lda);
}
hipError_t fl_set_identity(hipStream_t s, int64_t n, double* A, int64_t lda);
