// Kernels of the learned warm start: loop/star/harmonic coordinates and the
// perceptron (forward, backward, Adam).  gfx950: the products run on the
// 16x16x16 BF16 matrix cores with FP32 accumulation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "learned.h"

namespace qhp {

namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__device__ inline uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    uint32_t rounding = 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)((u + rounding) >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <int T>
__device__ inline uint16_t load_bf(const void *p, int64_t i)
{
    if constexpr (T == MT_BF16) return ((const uint16_t *)p)[i];
    else return f2bf(((const float *)p)[i]);
}

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

}  // namespace

// ------------------------------------------------------------ coordinates
__global__ void k_incidence_t(int64_t n, int64_t ne, int64_t nc, int64_t nv, const int32_t *tri_edge,
                              const int32_t *tri_sign, const int32_t *vedge_off, const int32_t *vedge,
                              const int32_t *edges, const double *Y, int64_t ldy, double *ysig, double *ylam)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t per = nc + nv;
    if (idx >= n * per) return;
    int64_t r = idx / per, q = idx % per;
    const double *y = Y + r * ldy;
    if (q < nc) {  // Sigma^T y: +1 where the cell is c+ of the edge
        double acc = 0.0;
        for (int j = 0; j < 3; ++j) acc += (double)tri_sign[3 * q + j] * y[tri_edge[3 * q + j]];
        ysig[r * nc + q] = acc;
    } else {  // Lambda^T y: +1 where the vertex is v+ of the edge
        int64_t v = q - nc;
        double acc = 0.0;
        for (int32_t e = vedge_off[v]; e < vedge_off[v + 1]; ++e) {
            int32_t ed = vedge[e];
            acc += edges[2 * ed + 1] == v ? y[ed] : -y[ed];
        }
        ylam[r * nv + v] = acc;
    }
}
void launch_incidence_t(hipStream_t s, int64_t n, int64_t ne, int64_t nc, int64_t nv, const int32_t *tri_edge,
                        const int32_t *tri_sign, const int32_t *vedge_off, const int32_t *vedge,
                        const int32_t *edges, const double *Y, int64_t ldy, double *ysig, double *ylam)
{
    hipLaunchKernelGGL(k_incidence_t, dim3(nblk(n * (nc + nv), 256)), dim3(256), 0, s, n, ne, nc, nv, tri_edge,
                       tri_sign, vedge_off, vedge, edges, Y, ldy, ysig, ylam);
}

__global__ void k_reconstruct(int64_t n, int64_t ne, int64_t nv, int64_t nc, int64_t nh, const int32_t *edges,
                              const int32_t *cells, const double *H, const double *F, int64_t ldf, double *Y,
                              int64_t ldy)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * ne) return;
    int64_t r = idx / ne, e = idx % ne;
    const double *f = F + r * ldf;
    double v = f[edges[2 * e + 1]] - f[edges[2 * e]];       // Lambda l
    v += f[nv + cells[2 * e]] - f[nv + cells[2 * e + 1]];   // Sigma s
    for (int64_t j = 0; j < nh; ++j) v += H[e * nh + j] * f[nv + nc + j];
    Y[r * ldy + e] = v;
}
void launch_reconstruct(hipStream_t s, int64_t n, int64_t ne, int64_t nv, int64_t nc, int64_t nh,
                        const int32_t *edges, const int32_t *cells, const double *H, const double *F, int64_t ldf,
                        double *Y, int64_t ldy)
{
    hipLaunchKernelGGL(k_reconstruct, dim3(nblk(n * ne, 256)), dim3(256), 0, s, n, ne, nv, nc, nh, edges, cells, H, F,
                       ldf, Y, ldy);
}

// ------------------------------------------------------------ products
// 64 x 64 output tile per work-group of four waves, each wave a 32 x 32
// quarter made of 2 x 2 MFMA 16x16x16 tiles; K staged through LDS in steps of
// 32 as BF16, both operands stored k-contiguous ([row][k] and [col][k]).
template <int TA, int TB>
__global__ __launch_bounds__(256) void k_mlp_gemm(int64_t M, int64_t N, int64_t K, float alpha, const void *A,
                                                  int64_t sam, int64_t sak, const void *B, int64_t sbk, int64_t sbn,
                                                  float beta, float *C, int64_t ldc, int64_t kchunk)
{
    constexpr int LDK = 40;  // 32 + 8 BF16 of padding per row
    __shared__ uint16_t As[64 * LDK];
    __shared__ uint16_t Bs[64 * LDK];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t m0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
    const int64_t kb = (int64_t)blockIdx.z * kchunk;
    const int64_t ke = min(K, kb + kchunk);
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    f4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    for (int64_t k0 = kb; k0 < ke; k0 += 32) {
        if (sak == 1) {  // A contiguous along k: 4 threads per row, 8 k each
            const int r = t >> 2, kk = (t & 3) * 8;
            const int64_t m = m0 + r;
            for (int i = 0; i < 8; ++i) {
                const int64_t k = k0 + kk + i;
                As[r * LDK + kk + i] = (m < M && k < ke) ? load_bf<TA>(A, m * sam + k) : (uint16_t)0;
            }
        } else {  // A contiguous along m: 8 threads per k, 8 rows each
            const int kk = t >> 3, r = (t & 7) * 8;
            const int64_t k = k0 + kk;
            for (int i = 0; i < 8; ++i) {
                const int64_t m = m0 + r + i;
                As[(r + i) * LDK + kk] = (m < M && k < ke) ? load_bf<TA>(A, m * sam + k * sak) : (uint16_t)0;
            }
        }
        if (sbk == 1) {  // B contiguous along k
            const int c = t >> 2, kk = (t & 3) * 8;
            const int64_t n = n0 + c;
            for (int i = 0; i < 8; ++i) {
                const int64_t k = k0 + kk + i;
                Bs[c * LDK + kk + i] = (n < N && k < ke) ? load_bf<TB>(B, k + n * sbn) : (uint16_t)0;
            }
        } else {  // B contiguous along n
            const int kk = t >> 3, c = (t & 7) * 8;
            const int64_t k = k0 + kk;
            for (int i = 0; i < 8; ++i) {
                const int64_t n = n0 + c + i;
                Bs[(c + i) * LDK + kk] = (n < N && k < ke) ? load_bf<TB>(B, k * sbk + n * sbn) : (uint16_t)0;
            }
        }
        __syncthreads();
        for (int ks = 0; ks < 32; ks += 16) {
            s4 a[2], b[2];
            const int ko = ks + 4 * (lane >> 4);
            for (int i = 0; i < 2; ++i) a[i] = *(const s4 *)&As[(wm + i * 16 + (lane & 15)) * LDK + ko];
            for (int j = 0; j < 2; ++j) b[j] = *(const s4 *)&Bs[(wn + j * 16 + (lane & 15)) * LDK + ko];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    const bool split = gridDim.z > 1;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 4; ++r) {
                const int64_t m = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
                const int64_t n = n0 + wn + j * 16 + (lane & 15);
                if (m >= M || n >= N) continue;
                const float v = alpha * acc[i][j][r];
                float *c = C + m * ldc + n;
                if (split) atomicAdd(c, v);
                else *c = beta == 0.f ? v : v + beta * *c;
            }
}

void mlp_gemm(hipStream_t s, int64_t M, int64_t N, int64_t K, float alpha, int ta, const void *A, int64_t sam,
              int64_t sak, int tb, const void *B, int64_t sbk, int64_t sbn, float beta, float *C, int64_t ldc,
              int ksplit)
{
    if (M <= 0 || N <= 0) return;
    ksplit = (int)std::max<int64_t>(1, std::min<int64_t>(ksplit, (K + 31) / 32));
    int64_t kchunk = (K + ksplit - 1) / ksplit;
    kchunk = (kchunk + 31) / 32 * 32;
    ksplit = (int)((K + kchunk - 1) / kchunk);
    dim3 grid(nblk(N, 64), nblk(M, 64), (unsigned)std::max(ksplit, 1));
#define QHP_GEMM(X, Y)                                                                                         \
    hipLaunchKernelGGL((k_mlp_gemm<X, Y>), grid, dim3(256), 0, s, M, N, K, alpha, A, sam, sak, B, sbk, sbn, beta, \
                       C, ldc, kchunk)
    if (ta == MT_BF16 && tb == MT_BF16) QHP_GEMM(MT_BF16, MT_BF16);
    else if (ta == MT_F32 && tb == MT_BF16) QHP_GEMM(MT_F32, MT_BF16);
    else if (ta == MT_F32 && tb == MT_F32) QHP_GEMM(MT_F32, MT_F32);
    else QHP_GEMM(MT_BF16, MT_F32);
#undef QHP_GEMM
}

// ------------------------------------------------------------ elementwise
__global__ void k_bias_tanh(int64_t rows, int64_t cols, const float *Z, const float *bias, float *A, uint16_t *Ab)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * cols) return;
    float a = tanhf(Z[i] + bias[i % cols]);
    A[i] = a;
    if (Ab) Ab[i] = f2bf(a);
}
void launch_bias_tanh(hipStream_t s, int64_t rows, int64_t cols, const float *Z, const float *bias, float *A,
                      uint16_t *Ab)
{
    hipLaunchKernelGGL(k_bias_tanh, dim3(nblk(rows * cols, 256)), dim3(256), 0, s, rows, cols, Z, bias, A, Ab);
}

__global__ void k_bias_add(int64_t rows, int64_t cols, float *Z, const float *bias)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < rows * cols) Z[i] += bias[i % cols];
}
void launch_bias_add(hipStream_t s, int64_t rows, int64_t cols, float *Z, const float *bias)
{
    hipLaunchKernelGGL(k_bias_add, dim3(nblk(rows * cols, 256)), dim3(256), 0, s, rows, cols, Z, bias);
}

__global__ void k_mse_grad(int64_t count, const float *O, const float *T, float *dO, double *loss_acc)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e2 = 0.0;
    if (i < count) {
        float e = O[i] - T[i];
        dO[i] = 2.f * e / (float)count;
        e2 = (double)e * (double)e;
    }
    for (int off = 32; off > 0; off >>= 1) e2 += __shfl_xor(e2, off, 64);
    __shared__ double part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = e2;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss_acc, (part[0] + part[1] + part[2] + part[3]) / (double)count);
}
void launch_mse_grad(hipStream_t s, int64_t count, const float *O, const float *T, float *dO, double *loss_acc)
{
    hipLaunchKernelGGL(k_mse_grad, dim3(nblk(count, 256)), dim3(256), 0, s, count, O, T, dO, loss_acc);
}

__global__ void k_tanh_back(int64_t count, const float *dA, const float *A, float *dZ)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dZ[i] = dA[i] * (1.f - A[i] * A[i]);
}
void launch_tanh_back(hipStream_t s, int64_t count, const float *dA, const float *A, float *dZ)
{
    hipLaunchKernelGGL(k_tanh_back, dim3(nblk(count, 256)), dim3(256), 0, s, count, dA, A, dZ);
}

__global__ void k_col_sum(int64_t rows, int64_t cols, const float *X, float *out)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    float acc = 0.f;
    for (int64_t i = 0; i < rows; ++i) acc += X[i * cols + j];
    out[j] = acc;
}
void launch_col_sum(hipStream_t s, int64_t rows, int64_t cols, const float *X, float *out)
{
    hipLaunchKernelGGL(k_col_sum, dim3(nblk(cols, 256)), dim3(256), 0, s, rows, cols, X, out);
}

__global__ void k_adam(int64_t count, float *w, const float *g, float *m, float *v, float lr_t, float b1, float b2,
                       float eps_t, uint16_t *wb)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float wi = w[i] - lr_t * mi / (sqrtf(vi) + eps_t);
    w[i] = wi;
    if (wb) wb[i] = f2bf(wi);
}
void launch_adam(hipStream_t s, int64_t count, float *w, const float *g, float *m, float *v, float lr_t, float b1,
                 float b2, float eps_t, uint16_t *wb)
{
    hipLaunchKernelGGL(k_adam, dim3(nblk(count, 256)), dim3(256), 0, s, count, w, g, m, v, lr_t, b1, b2, eps_t, wb);
}

__global__ void k_to_bf16(int64_t count, const float *x, uint16_t *y)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) y[i] = f2bf(x[i]);
}
void launch_to_bf16(hipStream_t s, int64_t count, const float *x, uint16_t *y)
{
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(count, 256)), dim3(256), 0, s, count, x, y);
}

__global__ void k_fill_f32(int64_t count, float value, float *x)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) x[i] = value;
}
void launch_fill_f32(hipStream_t s, int64_t count, float value, float *x)
{
    if (count > 0) hipLaunchKernelGGL(k_fill_f32, dim3(nblk(count, 256)), dim3(256), 0, s, count, value, x);
}
__global__ void k_fill_f64(int64_t count, double value, double *x)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) x[i] = value;
}
void launch_fill_f64(hipStream_t s, int64_t count, double value, double *x)
{
    if (count > 0) hipLaunchKernelGGL(k_fill_f64, dim3(nblk(count, 256)), dim3(256), 0, s, count, value, x);
}

// splitmix64 (Steele, Lea and Flood, OOPSLA 2014) of seed + counter
__device__ inline uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
__global__ void k_init_uniform(int64_t count, float a, uint64_t seed, uint64_t offset, float *w)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    uint64_t r = splitmix64(seed * 0x2545f4914f6cdd1dull + offset + (uint64_t)i);
    float u = (float)(r >> 40) * (1.0f / 16777216.0f);
    w[i] = a * (2.f * u - 1.f);
}
void launch_init_uniform(hipStream_t s, int64_t count, float a, uint64_t seed, uint64_t offset, float *w)
{
    if (count > 0)
        hipLaunchKernelGGL(k_init_uniform, dim3(nblk(count, 256)), dim3(256), 0, s, count, a, seed, offset, w);
}

// ------------------------------------------------------------ windows
__device__ inline double block_sum(double v, double *sh)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sh[q];
    return t;
}

__global__ void k_rms(int64_t n, int64_t nf, const double *F, double *sigma)
{
    __shared__ double sh[4];
    const double *f = F + (int64_t)blockIdx.x * nf;
    double acc = 0.0;
    for (int64_t q = threadIdx.x; q < nf; q += blockDim.x) acc += f[q] * f[q];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) sigma[blockIdx.x] = sqrt(acc / (double)nf);
}
void launch_rms(hipStream_t s, int64_t n, int64_t nf, const double *F, double *sigma)
{
    if (n > 0) hipLaunchKernelGGL(k_rms, dim3((unsigned)n), dim3(256), 0, s, n, nf, F, sigma);
}

// Backward differences of four consecutive feature rows f1 (newest) .. f4:
// d0 = f1, d1 = f1 - f2, d2 = f1 - 2 f2 + f3, d3 = f1 - 3 f2 + 3 f3 - f4,
// written as BF16(d_j / rms(d_j)) (a zero block stays 0); returns rms(d3).
__device__ double window_blocks(int64_t nf, const double *f1, const double *f2, const double *f3, const double *f4,
                                uint16_t *x)
{
    __shared__ double sh[4];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int64_t q = threadIdx.x; q < nf; q += blockDim.x) {
        const double a = f1[q], b = f2[q], c = f3[q], d = f4[q];
        const double d1 = a - b, d2 = a - 2.0 * b + c, d3 = a - 3.0 * b + 3.0 * c - d;
        s0 += a * a;
        s1 += d1 * d1;
        s2 += d2 * d2;
        s3 += d3 * d3;
    }
    double r[4] = {block_sum(s0, sh), block_sum(s1, sh), block_sum(s2, sh), block_sum(s3, sh)};
    double inv[4];
    for (int j = 0; j < 4; ++j) {
        r[j] = sqrt(r[j] / (double)nf);
        inv[j] = r[j] > 0.0 ? 1.0 / r[j] : 0.0;
    }
    for (int64_t q = threadIdx.x; q < nf; q += blockDim.x) {
        const double a = f1[q], b = f2[q], c = f3[q], d = f4[q];
        x[q] = f2bf((float)(a * inv[0]));
        x[nf + q] = f2bf((float)((a - b) * inv[1]));
        x[2 * nf + q] = f2bf((float)((a - 2.0 * b + c) * inv[2]));
        x[3 * nf + q] = f2bf((float)((a - 3.0 * b + 3.0 * c - d) * inv[3]));
    }
    return r[3];
}

__global__ void k_gather_windows(int64_t nf, const double *F, int64_t step, const int64_t *base, uint16_t *X, float *T)
{
    const int64_t b = blockIdx.x;
    const double *f1 = F + base[b] * nf, *f2 = f1 - step * nf, *f3 = f2 - step * nf, *f4 = f3 - step * nf;
    const double *f0 = f1 + step * nf;
    const double rho3 = window_blocks(nf, f1, f2, f3, f4, X + b * 4 * nf);
    const double inv = rho3 > 0.0 ? 1.0 / rho3 : 0.0;
    for (int64_t q = threadIdx.x; q < nf; q += blockDim.x)
        T[b * nf + q] = (float)((f0[q] - 3.0 * f1[q] + 3.0 * f2[q] - f3[q]) * inv);
}
void launch_gather_windows(hipStream_t s, int64_t B, int64_t nf, const double *F, int64_t step,
                           const int64_t *base, uint16_t *X, float *T)
{
    if (B > 0) hipLaunchKernelGGL(k_gather_windows, dim3((unsigned)B), dim3(256), 0, s, nf, F, step, base, X, T);
}

// rms of the third backward difference ending at each row (0 for rows < 3 step)
__global__ void k_rms_d3(int64_t nf, const double *F, int64_t step, double *out)
{
    __shared__ double sh[4];
    const int64_t r = blockIdx.x;
    if (r < 3 * step) {
        if (threadIdx.x == 0) out[r] = 0.0;
        return;
    }
    const double *f1 = F + r * nf, *f2 = f1 - step * nf, *f3 = f2 - step * nf, *f4 = f3 - step * nf;
    double acc = 0.0;
    for (int64_t q = threadIdx.x; q < nf; q += blockDim.x) {
        const double d3 = f1[q] - 3.0 * f2[q] + 3.0 * f3[q] - f4[q];
        acc += d3 * d3;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) out[r] = sqrt(acc / (double)nf);
}
void launch_rms_d3(hipStream_t s, int64_t rows, int64_t nf, const double *F, int64_t step, double *out)
{
    if (rows > 0) hipLaunchKernelGGL(k_rms_d3, dim3((unsigned)rows), dim3(256), 0, s, nf, F, step, out);
}

__global__ void k_window_x(int64_t nf, const double *f1, const double *f2, const double *f3, const double *f4,
                           uint16_t *X, double *rho3)
{
    const double r = window_blocks(nf, f1, f2, f3, f4, X);
    if (threadIdx.x == 0) *rho3 = r;
}
void launch_window_x(hipStream_t s, int64_t nf, const double *f1, const double *f2, const double *f3,
                     const double *f4, uint16_t *X, double *rho3)
{
    hipLaunchKernelGGL(k_window_x, dim3(1), dim3(256), 0, s, nf, f1, f2, f3, f4, X, rho3);
}

__global__ void k_guess(int64_t nf, const double *f1, const double *f2, const double *f3, const double *rho3,
                        const float *o, double *g)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nf) g[q] = 3.0 * f1[q] - 3.0 * f2[q] + f3[q] + *rho3 * (double)o[q];
}
void launch_guess(hipStream_t s, int64_t nf, const double *f1, const double *f2, const double *f3,
                  const double *rho3, const float *o, double *g)
{
    hipLaunchKernelGGL(k_guess, dim3(nblk(nf, 256)), dim3(256), 0, s, nf, f1, f2, f3, rho3, o, g);
}

}  // namespace qhp
