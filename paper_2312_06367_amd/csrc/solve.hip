// Per-step T_0 solve (marching scheme, Sec. IV-B: y_i = T_0^{-1} b_i) from
// the FP64 LU factors held in block-inverse form (see solve.h).
#include "solve.h"

#include <algorithm>
#include <cmath>

#include "linalg.h"
#include "march.h"

namespace qhp {

// D [rows][ld] = identity in its first rows x rows entries
__global__ void k_solve_eye(int64_t rows, int64_t ld, double *D)
{
    const int64_t n = rows * ld;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / ld, c = e % ld;
        D[e] = (r == c) ? 1.0 : 0.0;
    }
}

__global__ void k_solve_zero(int64_t n, double *p)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0.0;
}

// out[n][nrhs] rows gathered: out[i] = b[perm[i]]
__global__ void k_solve_gather(int64_t n, int64_t nrhs, const int32_t *perm, const double *b, double *out)
{
    const int64_t total = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / nrhs, j = e % nrhs;
        out[e] = b[(int64_t)perm[i] * nrhs + j];
    }
}

__device__ __forceinline__ double solve_dot(const double *__restrict__ a, const double *__restrict__ x, int64_t m,
                                            int tid)
{
    // 256 lanes over pairs of columns (16-byte loads of a row that starts on
    // an even element), a scalar tail when m is odd
    typedef double d2 __attribute__((ext_vector_type(2)));
    double s = 0.0;
    const int64_t mp = m & ~(int64_t)1;
#pragma unroll 4
    for (int64_t c = 2 * (int64_t)tid; c < mp; c += 512) {
        const d2 av = __builtin_nontemporal_load(reinterpret_cast<const d2 *>(a + c));
        const d2 xv = *reinterpret_cast<const d2 *>(x + c);
        s += av[0] * xv[0] + av[1] * xv[1];
    }
    if ((m & 1) && tid == 0) s += a[m - 1] * x[m - 1];
    return s;
}

// One row r of one block per work-group:
//   out[r] = sum_c D[r][c] xd[c] - sum_c Wr[r][c] xo[c]
// D: the block's diagonal inverse (row stride ldd, rows columns), xd its
// right-hand side (read through perm when perm is not null: xd[perm[pofs + c]]);
// Wr: the block's off-diagonal rows (row stride ldw, m columns), xo the
// solution pieces they multiply.
__global__ __launch_bounds__(256) void k_solve_row(int64_t rows, const double *__restrict__ D, int64_t ldd,
                                                   const double *__restrict__ xd, const int32_t *__restrict__ perm,
                                                   int64_t pofs, const double *__restrict__ Wr, int64_t ldw,
                                                   const double *__restrict__ xo, int64_t m, double *out)
{
    __shared__ double red[4];
    const int64_t r = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double s = 0.0;
    // diagonal-inverse part (rows <= kSolveBlock columns)
    if (perm) {
        for (int64_t c = tid; c < rows; c += 256) s += D[r * ldd + c] * xd[perm[pofs + c]];
    } else {
        s += solve_dot(D + r * ldd, xd, rows, tid);
    }
    if (m > 0) s -= solve_dot(Wr + r * ldw, xo, m, tid);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (tid == 0) out[r] = red[0] + red[1] + red[2] + red[3];
}

// partial[c][j] = sum of |A[i][j]| over the rows i of chunk c (kColChunks
// chunks); threads over columns, so every row is read coalesced
__global__ void k_col_abs_partial(int64_t n, const double *A, int64_t lda, int64_t rows_per_chunk, double *partial)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (j >= n) return;
    const int64_t i0 = c * rows_per_chunk, i1 = (i0 + rows_per_chunk < n) ? i0 + rows_per_chunk : n;
    double acc = 0.0;
    for (int64_t i = i0; i < i1; ++i) acc += fabs(A[i * lda + j]);
    partial[c * n + j] = acc;
}
// partial[c][j] = sum over the rows i of chunk c of A[i][j] x[i]  (A^T x)
__global__ void k_gemvT_partial(int64_t n, const double *A, int64_t lda, const double *x, int64_t rows_per_chunk,
                                double *partial)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (j >= n) return;
    const int64_t i0 = c * rows_per_chunk, i1 = (i0 + rows_per_chunk < n) ? i0 + rows_per_chunk : n;
    double acc = 0.0;
    for (int64_t i = i0; i < i1; ++i) acc += A[i * lda + j] * x[i];
    partial[c * n + j] = acc;
}
// out[j] = sum over the chunks c of partial[c][j] (in chunk order)
__global__ void k_chunk_sum(int64_t n, int nchunks, const double *partial, double *out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double acc = 0.0;
    for (int c = 0; c < nchunks; ++c) acc += partial[c * n + j];
    out[j] = acc;
}
// *out = |v|^2 (one work-group)
__global__ __launch_bounds__(1024) void k_sumsq(int64_t n, const double *v, double *out)
{
    __shared__ double red[16];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += v[i] * v[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        *out = t;
    }
}
// v = w / sqrt(*nrm2)
__global__ void k_scale_rsqrt(int64_t n, const double *w, const double *nrm2, double *v)
{
    const double f = 1.0 / sqrt(*nrm2);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = w[i] * f;
}
// a fixed start vector with no special direction
__global__ void k_power_start(int64_t n, double *v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = cos(0.7 * (double)i + 0.3) + 1.5;
}

void launch_col_abs_sums(hipStream_t s, int64_t n, const double *A, int64_t lda, double *partial, double *colsum)
{
    const int64_t rpc = (n + kColChunks - 1) / kColChunks;
    const unsigned gx = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_col_abs_partial, dim3(gx, (unsigned)kColChunks), dim3(256), 0, s, n, A, lda, rpc, partial);
    hipLaunchKernelGGL(k_chunk_sum, dim3(gx), dim3(256), 0, s, n, (int)kColChunks, partial, colsum);
}

double largest_singular_value(hipStream_t s, int64_t n, const double *A, int iters, double *work)
{
    double *v = work, *w = work + n, *t = work + 2 * n, *nrm = work + 3 * n, *partial = work + 3 * n + 8;
    const int64_t rpc = (n + kColChunks - 1) / kColChunks;
    const unsigned gx = (unsigned)((n + 255) / 256), gs = (unsigned)std::min<int64_t>(gx, 1024);
    hipLaunchKernelGGL(k_power_start, dim3(gs), dim3(256), 0, s, n, v);
    hipLaunchKernelGGL(k_sumsq, dim3(1), dim3(1024), 0, s, n, v, nrm);
    hipLaunchKernelGGL(k_scale_rsqrt, dim3(gs), dim3(256), 0, s, n, v, nrm, v);
    for (int it = 0; it < iters; ++it) {  // v <- A^T A v / |A^T A v|
        launch_gemv_f64(s, n, A, v, w);
        hipLaunchKernelGGL(k_gemvT_partial, dim3(gx, (unsigned)kColChunks), dim3(256), 0, s, n, A, n, w, rpc, partial);
        hipLaunchKernelGGL(k_chunk_sum, dim3(gx), dim3(256), 0, s, n, (int)kColChunks, partial, t);
        hipLaunchKernelGGL(k_sumsq, dim3(1), dim3(1024), 0, s, n, t, nrm);
        hipLaunchKernelGGL(k_scale_rsqrt, dim3(gs), dim3(256), 0, s, n, t, nrm, v);
    }
    double h = 0.0;
    if (hipMemcpyAsync(&h, nrm, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return -1.0;
    return std::sqrt(std::sqrt(h));  // |A^T A v| -> sigma_max^2 at convergence
}

void build_block_solve(hipStream_t s, int64_t n, const double *LU, int64_t lda, double *W, double *Dl, double *Du)
{
    const int64_t B = kSolveBlock, nb = (n + B - 1) / B, ldw = solve_ldw(n);
    hipLaunchKernelGGL(k_solve_zero, dim3(1024), dim3(256), 0, s, solve_w_elems(n), W);
    for (int64_t I = 0; I < nb; ++I) {
        const int64_t o = I * B, bi = std::min(B, n - o);
        double *dl = Dl + I * B * B, *du = Du + I * B * B;
        hipLaunchKernelGGL(k_solve_eye, dim3(256), dim3(256), 0, s, B, B, dl);
        hipLaunchKernelGGL(k_solve_eye, dim3(256), dim3(256), 0, s, B, B, du);
        trsm_f64(s, false, bi, bi, LU + o * lda + o, lda, dl, B);  // L_II^{-1}
        trsm_f64(s, true, bi, bi, LU + o * lda + o, lda, du, B);   // U_II^{-1}
        if (o > 0)  // W[I][0:o] = Dl_I L[I][0:o]
            gemm_f64(s, false, false, bi, o, bi, 1.0, dl, B, LU + o * lda, lda, 0.0, W + o * ldw, ldw);
        if (o + bi < n)  // W[I][o+bi:n] = Du_I U[I][o+bi:n]
            gemm_f64(s, false, false, bi, n - o - bi, bi, 1.0, du, B, LU + o * lda + o + bi, lda, 0.0,
                     W + o * ldw + o + bi, ldw);
    }
}

void launch_block_solve(hipStream_t s, int64_t n, int64_t nrhs, const double *W, const double *Dl,
                        const double *Du, const int32_t *perm, const double *b, double *z, double *y, double *work,
                        int64_t work_elems)
{
    const int64_t B = kSolveBlock, nb = (n + B - 1) / B, ldw = solve_ldw(n);
    if (nrhs == 1) {
        for (int64_t I = 0; I < nb; ++I) {  // z_I = Dl_I (P b)_I - W[I][0:o] z[0:o]
            const int64_t o = I * B, bi = std::min(B, n - o);
            hipLaunchKernelGGL(k_solve_row, dim3((unsigned)bi), dim3(256), 0, s, bi, Dl + I * B * B, B, b, perm, o,
                               W + o * ldw, ldw, z, o, z + o);
        }
        for (int64_t I = nb - 1; I >= 0; --I) {  // y_I = Du_I z_I - W[I][o+bi:n] y[o+bi:n]
            const int64_t o = I * B, bi = std::min(B, n - o), e = o + bi;
            hipLaunchKernelGGL(k_solve_row, dim3((unsigned)bi), dim3(256), 0, s, bi, Du + I * B * B, B, z + o,
                               (const int32_t *)nullptr, (int64_t)0, W + o * ldw + e, ldw, y + e, n - e, y + o);
        }
        return;
    }
    // several right-hand sides: the same blocks as matrix products; y holds
    // P b until the backward pass overwrites it block by block
    hipLaunchKernelGGL(k_solve_gather, dim3(1024), dim3(256), 0, s, n, nrhs, perm, b, y);
    for (int64_t I = 0; I < nb; ++I) {
        const int64_t o = I * B, bi = std::min(B, n - o);
        gemm_f64_splitk(s, bi, nrhs, bi, 1.0, Dl + I * B * B, B, y + o * nrhs, nrhs, 0.0, z + o * nrhs, nrhs, work,
                        work_elems);
        if (o > 0)
            gemm_f64_splitk(s, bi, nrhs, o, -1.0, W + o * ldw, ldw, z, nrhs, 1.0, z + o * nrhs, nrhs, work,
                            work_elems);
    }
    for (int64_t I = nb - 1; I >= 0; --I) {
        const int64_t o = I * B, bi = std::min(B, n - o), e = o + bi;
        gemm_f64_splitk(s, bi, nrhs, bi, 1.0, Du + I * B * B, B, z + o * nrhs, nrhs, 0.0, y + o * nrhs, nrhs, work,
                        work_elems);
        if (e < n)
            gemm_f64_splitk(s, bi, nrhs, n - e, -1.0, W + o * ldw + e, ldw, y + e * nrhs, nrhs, 1.0, y + o * nrhs,
                            nrhs, work, work_elems);
    }
}

}  // namespace qhp
