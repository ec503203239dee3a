// Kernels of the learned warm start: loop/star/harmonic coordinates of the
// solution vectors (the decomposition of Sec. II-D), a small tanh perceptron
// trained on the GPU (BF16 MFMA products, FP32 accumulation and master
// weights, Adam), and the iterative T_0 solve it warm-starts.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qhp {

// ---- loop/star/harmonic coordinates, FP64, vectors stored as rows
// Y [n][ldy] -> ysig [n][nc] = Sigma^T y, ylam [n][nv] = Lambda^T y
void launch_incidence_t(hipStream_t s, int64_t n, int64_t ne, int64_t nc, int64_t nv, const int32_t *tri_edge,
                        const int32_t *tri_sign, const int32_t *vedge_off, const int32_t *vedge,
                        const int32_t *edges, const double *Y, int64_t ldy, double *ysig, double *ylam);
// F [n][ldf] = [l | s | h] -> Y [n][ldy] = Lambda l + Sigma s + H h (H [ne][nh])
void launch_reconstruct(hipStream_t s, int64_t n, int64_t ne, int64_t nv, int64_t nc, int64_t nh,
                        const int32_t *edges, const int32_t *cells, const double *H, const double *F, int64_t ldf,
                        double *Y, int64_t ldy);

// ---- perceptron
enum { MT_F32 = 0, MT_BF16 = 1 };
// C[M][N] (row stride ldc, FP32) = alpha sum_k A(m,k) B(k,n) + beta C with
// A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn]; element types MT_F32 or
// MT_BF16, rounded to BF16 for the product, accumulated in FP32.  ksplit > 1
// splits K over work-groups that add atomically into C (beta ignored: the
// caller prepares C).
void mlp_gemm(hipStream_t s, int64_t M, int64_t N, int64_t K, float alpha, int ta, const void *A, int64_t sam,
              int64_t sak, int tb, const void *B, int64_t sbk, int64_t sbn, float beta, float *C, int64_t ldc,
              int ksplit);
// A = tanh(Z + bias) (rows x cols, bias per column); Ab = BF16(A) when non-null
void launch_bias_tanh(hipStream_t s, int64_t rows, int64_t cols, const float *Z, const float *bias, float *A,
                      uint16_t *Ab);
void launch_bias_add(hipStream_t s, int64_t rows, int64_t cols, float *Z, const float *bias);
// dO = 2 (O - T) / n; loss_acc += sum (O - T)^2 / n (n = count)
void launch_mse_grad(hipStream_t s, int64_t count, const float *O, const float *T, float *dO, double *loss_acc);
// dZ = dA (1 - A^2)
void launch_tanh_back(hipStream_t s, int64_t count, const float *dA, const float *A, float *dZ);
// out[j] = sum_i X[i][j]
void launch_col_sum(hipStream_t s, int64_t rows, int64_t cols, const float *X, float *out);
// Adam with the bias corrections folded into lr_t and eps_t; wb = BF16(w)
void launch_adam(hipStream_t s, int64_t count, float *w, const float *g, float *m, float *v, float lr_t, float b1,
                 float b2, float eps_t, uint16_t *wb);
void launch_to_bf16(hipStream_t s, int64_t count, const float *x, uint16_t *y);
void launch_fill_f32(hipStream_t s, int64_t count, float value, float *x);
void launch_fill_f64(hipStream_t s, int64_t count, double value, double *x);
// w[i] = a (2u - 1), u uniform in [0, 1) from splitmix64(seed, offset + i)
void launch_init_uniform(hipStream_t s, int64_t count, float a, uint64_t seed, uint64_t offset, float *w);
// per-row rms of F [n][nf] (FP64)
void launch_rms(hipStream_t s, int64_t n, int64_t nf, const double *F, double *sigma);
// training windows.  Sample b: rows r0 = base[b] of F (stride nf) with
// f_{i-1} at r0, f_{i-2} at r0 - step, ...; f_i at r0 + step.  With the
// backward differences d0 = f_{i-1}, d1, d2, d3 of f_{i-1..i-4}:
//   X[b] = BF16([d0 / rms(d0), d1 / rms(d1), d2 / rms(d2), d3 / rms(d3)])
//   T[b] = (f_i - 3 f_{i-1} + 3 f_{i-2} - f_{i-3}) / rms(d3) (FP32)
void launch_gather_windows(hipStream_t s, int64_t B, int64_t nf, const double *F, int64_t step,
                           const int64_t *base, uint16_t *X, float *T);
// rms(d3) of the window ending at each of `rows` rows (0 for rows < 3 step)
void launch_rms_d3(hipStream_t s, int64_t rows, int64_t nf, const double *F, int64_t step, double *out);
// one inference window from f1 = f_{i-1} .. f4 = f_{i-4}: X (BF16), rms(d3) (device)
void launch_window_x(hipStream_t s, int64_t nf, const double *f1, const double *f2, const double *f3,
                     const double *f4, uint16_t *X, double *rho3);
// guess of the next feature vector: g = 3 f1 - 3 f2 + f3 + rho3 o
void launch_guess(hipStream_t s, int64_t nf, const double *f1, const double *f2, const double *f3,
                  const double *rho3, const float *o, double *g);

// ---- iterative solve of T_0 (GMRES, FP32 Arnoldi, FP64 refinement)
// w = A v, A FP32 [n][lda], v and w FP32
void launch_gm_matvec(hipStream_t s, int64_t n, const float *A, int64_t lda, const float *v, float *w);
// h[q] += sum_i V[q][i] w[i] for q < nq (V rows of stride ldv), FP64 accumulators
void launch_gm_dots(hipStream_t s, int64_t n, int64_t nq, const float *V, int64_t ldv, const float *w, double *h);
// w -= sum_q h[q] V[q]; nrm2 += |w|^2 when nrm2 is non-null
void launch_gm_update(hipStream_t s, int64_t n, int64_t nq, const float *V, int64_t ldv, const double *h, float *w,
                      double *nrm2);
// Givens step of column j: Hcol[0..j] (from h1 + h2), h_{j+1,j} = sqrt(nrm2);
// rotations cs/sn [m], g [m+1], R column-major [m][m+1]; res = |g[j+1]|;
// inv = 1 / h_{j+1,j}; host_res (pinned) receives res.  h1, h2 (j + 2
// entries) and nrm2 are zeroed once read, ready for column j + 1.
void launch_gm_givens(hipStream_t s, int j, int m, double *h1, double *h2, double *nrm2, double *R, double *cs,
                      double *sn, double *g, double *inv, double *host_res);
// h1, h2 [m + 1] and nrm2 zeroed (before an inner solve's first column)
void launch_gm_clear(hipStream_t s, int m, double *h1, double *h2, double *nrm2);
// out = in * (*scale) (FP32 vector, FP64 scale)
void launch_gm_scale(hipStream_t s, int64_t n, const float *in, const double *scale, float *out);
// solve R y = g (k columns), x += sum_q y_q V[q] (x FP64)
void launch_gm_solution(hipStream_t s, int64_t n, int k, int m, const double *R, const double *g, double *ywork,
                        const float *V, int64_t ldv, double *x);
// r = b - A x (FP64, A [n][n]); nrm2 = |r|^2; v0 = r / |r| in FP32 is done by
// launch_gm_start once the norm is known
void launch_gm_residual(hipStream_t s, int64_t n, const double *A, const double *x, const double *b, double *r,
                        double *nrm2, double *host_nrm2);
void launch_gm_start(hipStream_t s, int64_t n, int m, const double *r, const double *nrm2, float *v0, double *g);
void launch_norm2(hipStream_t s, int64_t n, const double *x, double *nrm2, double *host);

}  // namespace qhp
