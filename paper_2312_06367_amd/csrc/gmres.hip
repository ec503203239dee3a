// Kernels of the iterative T_0 solve: restarted GMRES whose Arnoldi basis and
// products are FP32 (T_0 stored in FP32), inside an FP64 residual
// refinement loop, so the accepted solution meets an FP64 residual bound.
// Classical Gram-Schmidt with one re-orthogonalisation pass; the small
// Hessenberg least-squares problem is carried by Givens rotations in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "learned.h"

namespace qhp {

namespace {
inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
}  // namespace

// one wave per row, float4 loads along the row (lda % 4 == 0)
__global__ __launch_bounds__(256) void k_gm_matvec(int64_t n, const float *A, int64_t lda, const float *v, float *w)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const float *a = A + row * lda;
    float acc = 0.f;
    const int64_t n4 = n / 4 * 4;
    for (int64_t c = 4 * lane; c < n4; c += 256) {
        float4 x = *(const float4 *)(a + c);
        float4 y = *(const float4 *)(v + c);
        acc += x.x * y.x + x.y * y.y + x.z * y.z + x.w * y.w;
    }
    for (int64_t c = n4 + lane; c < n; c += 64) acc += a[c] * v[c];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) w[row] = acc;
}
void launch_gm_matvec(hipStream_t s, int64_t n, const float *A, int64_t lda, const float *v, float *w)
{
    hipLaunchKernelGGL(k_gm_matvec, dim3(nblk(n, 4)), dim3(256), 0, s, n, A, lda, v, w);
}

// partial dot products of a row chunk with every basis vector; one FP64
// atomic per (block, q)
__global__ __launch_bounds__(256) void k_gm_dots(int64_t n, int64_t nq, const float *V, int64_t ldv, const float *w,
                                                  double *h)
{
    __shared__ double sh[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const float wi = i < n ? w[i] : 0.f;
    for (int64_t q = 0; q < nq; ++q) {
        double p = i < n ? (double)V[q * ldv + i] * (double)wi : 0.0;
        for (int off = 32; off > 0; off >>= 1) p += __shfl_xor(p, off, 64);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = p;
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(&h[q], sh[0] + sh[1] + sh[2] + sh[3]);
    }
}
void launch_gm_dots(hipStream_t s, int64_t n, int64_t nq, const float *V, int64_t ldv, const float *w, double *h)
{
    hipLaunchKernelGGL(k_gm_dots, dim3(nblk(n, 256)), dim3(256), 0, s, n, nq, V, ldv, w, h);
}

__global__ __launch_bounds__(256) void k_gm_update(int64_t n, int64_t nq, const float *V, int64_t ldv,
                                                    const double *h, float *w, double *nrm2)
{
    __shared__ double sh[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double x = 0.0;
    if (i < n) {
        double acc = (double)w[i];
        for (int64_t q = 0; q < nq; ++q) acc -= h[q] * (double)V[q * ldv + i];
        w[i] = (float)acc;
        x = (double)(float)acc;
        x *= x;
    }
    if (!nrm2) return;
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(nrm2, sh[0] + sh[1] + sh[2] + sh[3]);
}
void launch_gm_update(hipStream_t s, int64_t n, int64_t nq, const float *V, int64_t ldv, const double *h, float *w,
                      double *nrm2)
{
    hipLaunchKernelGGL(k_gm_update, dim3(nblk(n, 256)), dim3(256), 0, s, n, nq, V, ldv, h, w, nrm2);
}

// R is column-major with leading dimension m + 1: R[q + j (m + 1)].  The
// accumulators h1, h2 (j + 2 entries) and nrm2 are left zero for iteration
// j + 1 once read.
__global__ void k_gm_givens(int j, int m, double *h1, double *h2, double *nrm2, double *R, double *cs, double *sn,
                            double *g, double *inv, double *host_res)
{
    if (threadIdx.x != 0) return;
    double *col = R + (int64_t)j * (m + 1);
    for (int q = 0; q <= j; ++q) col[q] = h1[q] + h2[q];
    double hn = sqrt(*nrm2);
    for (int q = 0; q <= j + 1 && q <= m; ++q) h1[q] = h2[q] = 0.0;
    *nrm2 = 0.0;
    col[j + 1] = hn;
    for (int q = 0; q < j; ++q) {  // earlier rotations
        double a = col[q], b = col[q + 1];
        col[q] = cs[q] * a + sn[q] * b;
        col[q + 1] = -sn[q] * a + cs[q] * b;
    }
    double a = col[j], b = col[j + 1];
    double r = hypot(a, b);
    double c = r > 0.0 ? a / r : 1.0, sv = r > 0.0 ? b / r : 0.0;
    cs[j] = c;
    sn[j] = sv;
    col[j] = r;
    col[j + 1] = 0.0;
    double gj = g[j];
    g[j] = c * gj;
    g[j + 1] = -sv * gj;
    *inv = hn > 0.0 ? 1.0 / hn : 0.0;
    *host_res = fabs(g[j + 1]);
}
void launch_gm_givens(hipStream_t s, int j, int m, double *h1, double *h2, double *nrm2, double *R, double *cs,
                      double *sn, double *g, double *inv, double *host_res)
{
    hipLaunchKernelGGL(k_gm_givens, dim3(1), dim3(64), 0, s, j, m, h1, h2, nrm2, R, cs, sn, g, inv, host_res);
}

// zero the Arnoldi accumulators h1, h2 (m + 1 entries each) and nrm2 before
// an inner solve's first iteration
__global__ void k_gm_clear(int m, double *h1, double *h2, double *nrm2)
{
    for (int q = threadIdx.x; q <= m; q += blockDim.x) h1[q] = h2[q] = 0.0;
    if (threadIdx.x == 0) *nrm2 = 0.0;
}
void launch_gm_clear(hipStream_t s, int m, double *h1, double *h2, double *nrm2)
{
    hipLaunchKernelGGL(k_gm_clear, dim3(1), dim3(64), 0, s, m, h1, h2, nrm2);
}

__global__ void k_gm_scale(int64_t n, const float *in, const double *scale, float *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)((double)in[i] * *scale);
}
void launch_gm_scale(hipStream_t s, int64_t n, const float *in, const double *scale, float *out)
{
    hipLaunchKernelGGL(k_gm_scale, dim3(nblk(n, 256)), dim3(256), 0, s, n, in, scale, out);
}

// back substitution on the rotated Hessenberg (one wave), then x += V y
__global__ void k_gm_backsolve(int k, int m, const double *R, const double *g, double *y)
{
    if (threadIdx.x != 0) return;
    for (int q = k - 1; q >= 0; --q) {
        double acc = g[q];
        for (int p = q + 1; p < k; ++p) acc -= R[q + (int64_t)p * (m + 1)] * y[p];
        double d = R[q + (int64_t)q * (m + 1)];
        y[q] = d != 0.0 ? acc / d : 0.0;
    }
}
__global__ void k_gm_combine(int64_t n, int k, const double *y, const float *V, int64_t ldv, double *x)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int q = 0; q < k; ++q) acc += y[q] * (double)V[q * ldv + i];
    x[i] += acc;
}
void launch_gm_solution(hipStream_t s, int64_t n, int k, int m, const double *R, const double *g, double *ywork,
                        const float *V, int64_t ldv, double *x)
{
    if (k <= 0) return;
    hipLaunchKernelGGL(k_gm_backsolve, dim3(1), dim3(64), 0, s, k, m, R, g, ywork);
    hipLaunchKernelGGL(k_gm_combine, dim3(nblk(n, 256)), dim3(256), 0, s, n, k, ywork, V, ldv, x);
}

// r = b - A x (FP64 row per wave), |r|^2 accumulated
__global__ __launch_bounds__(256) void k_gm_residual(int64_t n, const double *A, const double *x, const double *b,
                                                      double *r, double *nrm2)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    double acc = 0.0;
    if (row < n) {
        const double *a = A + row * n;
        for (int64_t c = lane; c < n; c += 64) acc += a[c] * x[c];
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __shared__ double sh[4];
    if (lane == 0) {
        double ri = row < n ? b[row] - acc : 0.0;
        if (row < n) r[row] = ri;
        sh[threadIdx.x >> 6] = ri * ri;
    }
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(nrm2, sh[0] + sh[1] + sh[2] + sh[3]);
}
__global__ void k_copy_scalar(const double *src, double *dst)
{
    if (threadIdx.x == 0) *dst = *src;
}
void launch_gm_residual(hipStream_t s, int64_t n, const double *A, const double *x, const double *b, double *r,
                        double *nrm2, double *host_nrm2)
{
    launch_fill_f64(s, 1, 0.0, nrm2);
    hipLaunchKernelGGL(k_gm_residual, dim3(nblk(n, 4)), dim3(256), 0, s, n, A, x, b, r, nrm2);
    if (host_nrm2) hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(64), 0, s, nrm2, host_nrm2);
}

// v0 = r / |r| (FP32), g = (|r|, 0, ..., 0)
__global__ void k_gm_start(int64_t n, int m, const double *r, const double *nrm2, float *v0, double *g)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double beta = sqrt(*nrm2);
    const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
    if (i < n) v0[i] = (float)(r[i] * inv);
    if (i <= m) g[i] = i == 0 ? beta : 0.0;
}
void launch_gm_start(hipStream_t s, int64_t n, int m, const double *r, const double *nrm2, float *v0, double *g)
{
    hipLaunchKernelGGL(k_gm_start, dim3(nblk(std::max<int64_t>(n, m + 1), 256)), dim3(256), 0, s, n, m, r, nrm2, v0,
                       g);
}

__global__ void k_norm2(int64_t n, const double *x, double *nrm2)
{
    __shared__ double sh[4];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = i < n ? x[i] * x[i] : 0.0;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(nrm2, sh[0] + sh[1] + sh[2] + sh[3]);
}
void launch_norm2(hipStream_t s, int64_t n, const double *x, double *nrm2, double *host)
{
    launch_fill_f64(s, 1, 0.0, nrm2);
    hipLaunchKernelGGL(k_norm2, dim3(nblk(n, 256)), dim3(256), 0, s, n, x, nrm2);
    if (host) hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(64), 0, s, nrm2, host);
}

}  // namespace qhp
