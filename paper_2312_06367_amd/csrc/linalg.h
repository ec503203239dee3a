// Dense FP64 building blocks used by the one-time assembly (row-major).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qhp {

// C = alpha op(A) op(B) + beta C; op(A) is M x K, op(B) is K x N.
void gemm_f64(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
              const double *A, int64_t lda, const double *B, int64_t ldb, double beta, double *C,
              int64_t ldc);
// C = alpha A B + beta C (no transposes) with k split over extra work-groups
// when the tile grid alone would not fill the chip: work holds work_elems
// doubles of partial products (at least 2 M N for a split), summed in a fixed
// order; without room it is gemm_f64.
void gemm_f64_splitk(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, const double *A, int64_t lda,
                     const double *B, int64_t ldb, double beta, double *C, int64_t ldc, double *work,
                     int64_t work_elems);
void scale_f64(hipStream_t s, int64_t M, int64_t N, double beta, double *C, int64_t ldc);
void eye_plus(hipStream_t s, int64_t n, double a, double b, const double *P, double *out);
void axpby(hipStream_t s, int64_t n, double a, const double *x, double b, const double *y, double *out);
void transpose_f64(hipStream_t s, int64_t rows, int64_t cols, const double *in, int64_t ldi,
                   double *out, int64_t ldo);
void symmetrize(hipStream_t s, int64_t n, double *A);
// count += number of nonzero entries of x [n] (device counter)
void count_nonzero(hipStream_t s, int64_t n, const double *x, unsigned long long *count);
// In-place LU with partial pivoting (P A = L U, unit L); ipiv is device
// [n] (0-based row swapped with row j at step j).  Returns 0 or j+1 of the
// first zero pivot.  Synchronises the stream.
int getrf_f64(hipStream_t s, int64_t n, double *A, int64_t lda, int32_t *ipiv, int *info_dev);
// Solve T X = B for the unit lower (upper = false) or the upper (upper =
// true) triangle T of an n x n LU factor, no pivoting; B [n][nrhs] overwritten.
void trsm_f64(hipStream_t s, bool upper, int64_t n, int64_t nrhs, const double *T, int64_t lda, double *B,
              int64_t ldb);
// Solve A X = B (trans = false) or A^T X = B, B [n][nrhs] overwritten.
void getrs_f64(hipStream_t s, bool trans, int64_t n, int64_t nrhs, const double *LU, int64_t lda,
               const int32_t *ipiv, double *B, int64_t ldb);

}  // namespace qhp
