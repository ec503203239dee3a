// Per-step T_0 solve from the LU factors in block-inverse form.
//
// With P T_0 = L U (unit L) and diagonal blocks of kSolveBlock rows, the
// factors are kept as Dl_I = L_II^{-1}, Du_I = U_II^{-1} and one n x n matrix
// W whose strictly lower blocks are W_IJ = Dl_I L_IJ (J < I) and whose strictly
// upper blocks are W_IJ = Du_I U_IJ (J > I).  Then
//   z_I = Dl_I (P b)_I - sum_{J<I} W_IJ z_J     (I = 0, 1, ...)
//   y_I = Du_I z_I     - sum_{J>I} W_IJ y_J     (I = last, ..., 0)
// is the same pair of triangular solves: each block is one product over
// memory that is ready, so a solve is 2 n / kSolveBlock launches rather than a
// chain of dependent 64-row steps.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qhp {

constexpr int64_t kSolveBlock = 1024;

// row stride of W (n rounded up to an even count: 16-byte loads)
inline int64_t solve_ldw(int64_t n) { return (n + 1) / 2 * 2; }
// elements of W and of each of Dl, Du ([nblocks][kSolveBlock][kSolveBlock])
inline int64_t solve_w_elems(int64_t n) { return n * solve_ldw(n); }
inline int64_t solve_d_elems(int64_t n) { return (n + kSolveBlock - 1) / kSolveBlock * kSolveBlock * kSolveBlock; }

// LU (n x n, row stride lda, from getrf_f64) -> W, Dl, Du (device buffers of
// the sizes above).  Synchronises nothing; work is on stream s.
void build_block_solve(hipStream_t s, int64_t n, const double *LU, int64_t lda, double *W, double *Dl, double *Du);

// y = T_0^{-1} b for b, y [n][nrhs] (nrhs >= 1); z [n][nrhs] is scratch,
// work (work_elems doubles, may be null) room for the split-k partial
// products of the several-right-hand-side form.  perm[i] is the row of b that
// becomes row i of P b.
void launch_block_solve(hipStream_t s, int64_t n, int64_t nrhs, const double *W, const double *Dl,
                        const double *Du, const int32_t *perm, const double *b, double *z, double *y, double *work,
                        int64_t work_elems);

// column sums of |A| (n x n, row stride lda) into colsum [n]; partial holds
// kColChunks * n doubles (fixed summation order)
constexpr int64_t kColChunks = 32;
void launch_col_abs_sums(hipStream_t s, int64_t n, const double *A, int64_t lda, double *partial, double *colsum);
// doubles of work for largest_singular_value
inline int64_t power_work_elems(int64_t n) { return 3 * n + 8 + kColChunks * n; }
// largest singular value of A (n x n, row stride n) by iters steps of power
// iteration on A^T A from a fixed start vector; work holds
// power_work_elems(n) doubles.  Synchronises the stream; -1 on a device error.
double largest_singular_value(hipStream_t s, int64_t n, const double *A, int iters, double *work);

}  // namespace qhp
