// Dense FP64 linear algebra on gfx950 for the one-time assembly: MFMA GEMM,
// LU with partial pivoting and triangular solves with many right-hand sides.
// All matrices are row-major with an explicit leading dimension.
#include "linalg.h"

#include <algorithm>
#include <vector>

namespace qhp {

typedef double d4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ GEMM
// C = alpha op(A) op(B) + beta C.  64x64 block tile, k-tile 16, four waves
// each owning a 32x32 quadrant made of 2x2 v_mfma_f64_16x16x4 tiles.  With
// work set, work-group z covers k in [z kchunk, (z + 1) kchunk) and writes
// alpha times its partial product to work[z] ([M][N]); beta is then unused.
// MFMA operands: lane l holds A[l%16][l/16] and B[l/16][l%16]; the result
// lane l, register r holds D[4*r + l/16][l%16] (checked on gfx950).
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_f64(int64_t M, int64_t N, int64_t K, double alpha,
                                                  const double *__restrict__ A, int64_t lda,
                                                  const double *__restrict__ B, int64_t ldb,
                                                  double beta, double *__restrict__ C, int64_t ldc,
                                                  int64_t kchunk, double *__restrict__ work)
{
    __shared__ double As[2][16][66];
    const int64_t kb = (int64_t)blockIdx.z * kchunk;
    const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
    __shared__ double Bs[2][16][66];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    d4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

    double ra[4], rb[4];
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int e = tid + 256 * q;
            int ii, kk;
            if (!TA) { ii = e >> 4; kk = e & 15; } else { kk = e >> 6; ii = e & 63; }
            int64_t gi = i0 + ii, gk = k0 + kk;
            ra[q] = (gi < M && gk < ke) ? (TA ? A[gk * lda + gi] : A[gi * lda + gk]) : 0.0;
            int jj;
            if (!TB) { kk = e >> 6; jj = e & 63; } else { jj = e >> 4; kk = e & 15; }
            int64_t gj = j0 + jj;
            gk = k0 + kk;
            rb[q] = (gk < ke && gj < N) ? (TB ? B[gj * ldb + gk] : B[gk * ldb + gj]) : 0.0;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int e = tid + 256 * q;
            int ii, kk, jj;
            if (!TA) { ii = e >> 4; kk = e & 15; } else { kk = e >> 6; ii = e & 63; }
            As[buf][kk][ii] = ra[q];
            if (!TB) { kk = e >> 6; jj = e & 63; } else { jj = e >> 4; kk = e & 15; }
            Bs[buf][kk][jj] = rb[q];
        }
    };
    int buf = 0;
    gload(kb);
    sstore(0);
    __syncthreads();
    for (int64_t k0 = kb; k0 < ke; k0 += 16) {
        const bool more = k0 + 16 < ke;
        if (more) gload(k0 + 16);
#pragma unroll
        for (int kq = 0; kq < 16; kq += 4) {
            int kk = kq + (lane >> 4);
            double a0 = As[buf][kk][wi + (lane & 15)];
            double a1 = As[buf][kk][wi + 16 + (lane & 15)];
            double b0 = Bs[buf][kk][wj + (lane & 15)];
            double b1 = Bs[buf][kk][wj + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        if (more) {
            sstore(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int64_t gi = i0 + wi + 16 * ti + 4 * r + (lane >> 4);
                int64_t gj = j0 + wj + 16 * tj + (lane & 15);
                if (gi < M && gj < N) {
                    double v = alpha * acc[ti][tj][r];
                    if (work) {
                        work[((int64_t)blockIdx.z * M + gi) * N + gj] = v;
                    } else {
                        if (beta != 0.0) v += beta * C[gi * ldc + gj];
                        C[gi * ldc + gj] = v;
                    }
                }
            }
}

void gemm_f64(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
              const double *A, int64_t lda, const double *B, int64_t ldb, double beta, double *C,
              int64_t ldc)
{
    if (M <= 0 || N <= 0) return;
    if (K <= 0) {
        scale_f64(s, M, N, beta, C, ldc);
        return;
    }
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
    double *nw = nullptr;
    if (!ta && !tb) hipLaunchKernelGGL((k_gemm_f64<false, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, K, nw);
    else if (ta && !tb) hipLaunchKernelGGL((k_gemm_f64<true, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, K, nw);
    else if (!ta && tb) hipLaunchKernelGGL((k_gemm_f64<false, true>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, K, nw);
    else hipLaunchKernelGGL((k_gemm_f64<true, true>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, K, nw);
}

// C = beta C + sum_z work[z] (z = 0, 1, ... in order)
__global__ void k_splitk_sum(int64_t M, int64_t N, int nz, const double *work, double beta, double *C, int64_t ldc)
{
    const int64_t n = M * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int z = 0; z < nz; ++z) v += work[z * n + e];
        const int64_t i = e / N, j = e % N;
        if (beta != 0.0) v += beta * C[i * ldc + j];
        C[i * ldc + j] = v;
    }
}

void gemm_f64_splitk(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, const double *A, int64_t lda,
                     const double *B, int64_t ldb, double beta, double *C, int64_t ldc, double *work,
                     int64_t work_elems)
{
    if (M <= 0 || N <= 0) return;
    const int64_t tiles = ((N + 63) / 64) * ((M + 63) / 64);
    // enough work-groups for two per CU (256 CUs), k-ranges of at least 256
    int64_t nz = std::min<int64_t>((512 + tiles - 1) / tiles, K / 256);
    nz = std::min<int64_t>(nz, work_elems / (M * N));
    if (nz < 2 || !work) return gemm_f64(s, false, false, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    const int64_t kchunk = ((K + nz - 1) / nz + 15) / 16 * 16;
    nz = (K + kchunk - 1) / kchunk;
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)nz);
    hipLaunchKernelGGL((k_gemm_f64<false, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, 0.0, C,
                       ldc, kchunk, work);
    const int64_t n = M * N;
    hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 2048)), dim3(256), 0, s, M, N,
                       (int)nz, work, beta, C, ldc);
}

// ------------------------------------------------------------ elementwise
__global__ void k_scale(int64_t M, int64_t N, double beta, double *C, int64_t ldc)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * N) return;
    int64_t i = idx / N, j = idx % N;
    C[i * ldc + j] = beta == 0.0 ? 0.0 : beta * C[i * ldc + j];
}
void scale_f64(hipStream_t s, int64_t M, int64_t N, double beta, double *C, int64_t ldc)
{
    int64_t n = M * N;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, M, N, beta, C, ldc);
}

// out = a * I + b * P  (n x n)
__global__ void k_eye_plus(int64_t n, double a, double b, const double *P, double *out)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    int64_t i = idx / n, j = idx % n;
    out[idx] = b * P[idx] + (i == j ? a : 0.0);
}
void eye_plus(hipStream_t s, int64_t n, double a, double b, const double *P, double *out)
{
    hipLaunchKernelGGL(k_eye_plus, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, n, a, b, P, out);
}

// out = a x + b y
__global__ void k_axpby(int64_t n, double a, const double *x, double b, const double *y, double *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}
void axpby(hipStream_t s, int64_t n, double a, const double *x, double b, const double *y, double *out)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a, x, b, y, out);
}

// out[j][i] = in[i][j], in is rows x cols
__global__ void k_transpose(int64_t rows, int64_t cols, const double *in, int64_t ldi, double *out, int64_t ldo)
{
    __shared__ double tile[32][33];
    int64_t bi = (int64_t)blockIdx.y * 32, bj = (int64_t)blockIdx.x * 32;
    int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        int64_t i = bi + r, j = bj + tx;
        if (i < rows && j < cols) tile[r][tx] = in[i * ldi + j];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        int64_t j = bj + r, i = bi + tx;
        if (i < rows && j < cols) out[j * ldo + i] = tile[tx][r];
    }
}
void transpose_f64(hipStream_t s, int64_t rows, int64_t cols, const double *in, int64_t ldi, double *out, int64_t ldo)
{
    dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
    hipLaunchKernelGGL(k_transpose, grid, dim3(32, 8), 0, s, rows, cols, in, ldi, out, ldo);
}

// A = (A + A^T) / 2 (square n)
__global__ void k_symmetrize(int64_t n, double *A)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    int64_t i = idx / n, j = idx % n;
    if (j <= i) return;
    double v = 0.5 * (A[i * n + j] + A[j * n + i]);
    A[i * n + j] = v;
    A[j * n + i] = v;
}
void symmetrize(hipStream_t s, int64_t n, double *A)
{
    hipLaunchKernelGGL(k_symmetrize, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, n, A);
}

// ------------------------------------------------------------------- LU
// Panel factorisation of columns [j0, j0+nb) over rows [j0, n) by one
// workgroup: pivot search, row swap inside the panel, scaling, rank-1 update.
__global__ __launch_bounds__(1024) void k_panel(int64_t n, int64_t j0, int nb, double *A, int64_t lda,
                                                int32_t *ipiv, int *info)
{
    __shared__ double sval[1024];
    __shared__ int64_t sidx[1024];
    __shared__ double prow[64];
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int jj = 0; jj < nb; ++jj) {
        int64_t j = j0 + jj;
        double best = -1.0;
        int64_t bi = j;
        for (int64_t i = j + tid; i < n; i += nt) {
            double v = fabs(A[i * lda + j]);
            if (v > best) { best = v; bi = i; }
        }
        sval[tid] = best;
        sidx[tid] = bi;
        __syncthreads();
        for (int off = nt / 2; off > 0; off >>= 1) {
            if (tid < off) {
                double o = sval[tid + off];
                int64_t oi = sidx[tid + off];
                if (o > sval[tid] || (o == sval[tid] && oi < sidx[tid])) { sval[tid] = o; sidx[tid] = oi; }
            }
            __syncthreads();
        }
        int64_t p = sidx[0];
        double pv = sval[0];
        __syncthreads();
        if (tid == 0) {
            ipiv[j] = (int32_t)p;
            if (!(pv > 0.0) && *info == 0) *info = (int)(j + 1);
        }
        // swap rows j and p over the panel columns
        if (p != j && tid < nb) {
            double t = A[j * lda + j0 + tid];
            A[j * lda + j0 + tid] = A[p * lda + j0 + tid];
            A[p * lda + j0 + tid] = t;
        }
        __syncthreads();
        if (tid < nb) prow[tid] = A[j * lda + j0 + tid];
        __syncthreads();
        double piv = prow[jj];
        double inv = (piv != 0.0) ? 1.0 / piv : 0.0;
        for (int64_t i = j + 1 + tid; i < n; i += nt) {
            double l = A[i * lda + j] * inv;
            A[i * lda + j] = l;
            for (int c = jj + 1; c < nb; ++c) A[i * lda + j0 + c] -= l * prow[c];
        }
        __syncthreads();
    }
}

// apply the panel's row interchanges to columns outside [j0, j0+nb)
__global__ void k_laswp(int64_t n, int64_t j0, int nb, double *A, int64_t lda, const int32_t *ipiv)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n - nb) return;
    int64_t col = c < j0 ? c : c + nb;
    for (int jj = 0; jj < nb; ++jj) {
        int64_t j = j0 + jj, p = ipiv[j];
        if (p != j) {
            double t = A[j * lda + col];
            A[j * lda + col] = A[p * lda + col];
            A[p * lda + col] = t;
        }
    }
}

// U12 = L11^{-1} A12 for the nb x (n - j0 - nb) block right of the panel
__global__ __launch_bounds__(256) void k_trsm_row(int64_t n, int64_t j0, int nb, double *A, int64_t lda)
{
    __shared__ double L[64][65];
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
        int r = e / nb, c = e % nb;
        L[r][c] = A[(j0 + r) * lda + j0 + c];
    }
    __syncthreads();
    int64_t col = j0 + nb + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= n) return;
    double x[64];
    for (int r = 0; r < nb; ++r) {
        double v = A[(j0 + r) * lda + col];
        for (int c = 0; c < r; ++c) v -= L[r][c] * x[c];
        x[r] = v;
    }
    for (int r = 0; r < nb; ++r) A[(j0 + r) * lda + col] = x[r];
}

int getrf_f64(hipStream_t s, int64_t n, double *A, int64_t lda, int32_t *ipiv, int *info_dev)
{
    const int NB = 32;
    (void)hipMemsetAsync(info_dev, 0, sizeof(int), s);
    for (int64_t j0 = 0; j0 < n; j0 += NB) {
        int nb = (int)std::min<int64_t>(NB, n - j0);
        hipLaunchKernelGGL(k_panel, dim3(1), dim3(1024), 0, s, n, j0, nb, A, lda, ipiv, info_dev);
        if (n - nb > 0)
            hipLaunchKernelGGL(k_laswp, dim3((unsigned)((n - nb + 255) / 256)), dim3(256), 0, s, n, j0, nb, A, lda, ipiv);
        int64_t rest = n - j0 - nb;
        if (rest > 0) {
            hipLaunchKernelGGL(k_trsm_row, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0, s, n, j0, nb, A, lda);
            gemm_f64(s, false, false, rest, rest, nb, -1.0, A + (j0 + nb) * lda + j0, lda,
                     A + j0 * lda + j0 + nb, lda, 1.0, A + (j0 + nb) * lda + j0 + nb, lda);
        }
    }
    int info = 0;
    (void)hipMemcpyAsync(&info, info_dev, sizeof(int), hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
    return info;
}

// --------------------------------------------------------------- solves
// Row interchanges on B [n][nrhs] (forward or reverse order).
__global__ void k_rowswap(int64_t n, int64_t nrhs, double *B, int64_t ldb, const int32_t *ipiv, int reverse)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrhs) return;
    for (int64_t q = 0; q < n; ++q) {
        int64_t j = reverse ? n - 1 - q : q;
        int64_t p = ipiv[j];
        if (p != j) {
            double t = B[j * ldb + c];
            B[j * ldb + c] = B[p * ldb + c];
            B[p * ldb + c] = t;
        }
    }
}

// Solve a small triangular block in place: B[b0:b0+nb, :] = op(T)^{-1} B[...].
// mode: 0 = L unit lower, 1 = U non-unit upper, 2 = U^T (lower, non-unit),
// 3 = L^T (upper, unit); T is the nb x nb diagonal block at LU[b0][b0].
__global__ __launch_bounds__(256) void k_trsm_blk(int64_t b0, int nb, const double *LU, int64_t lda,
                                                  double *B, int64_t ldb, int64_t nrhs, int mode)
{
    __shared__ double T[64][65];
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
        int r = e / nb, c = e % nb;
        double v = LU[(b0 + r) * lda + b0 + c];
        if (mode >= 2) T[c][r] = v; else T[r][c] = v;  // transpose for U^T / L^T
    }
    __syncthreads();
    int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= nrhs) return;
    double x[64];
    bool lower = (mode == 0 || mode == 2);
    bool unit = (mode == 0 || mode == 3);
    if (lower) {
        for (int r = 0; r < nb; ++r) {
            double v = B[(b0 + r) * ldb + col];
            for (int c = 0; c < r; ++c) v -= T[r][c] * x[c];
            x[r] = unit ? v : v / T[r][r];
        }
    } else {
        for (int r = nb - 1; r >= 0; --r) {
            double v = B[(b0 + r) * ldb + col];
            for (int c = r + 1; c < nb; ++c) v -= T[r][c] * x[c];
            x[r] = unit ? v : v / T[r][r];
        }
    }
    for (int r = 0; r < nb; ++r) B[(b0 + r) * ldb + col] = x[r];
}

void trsm_f64(hipStream_t s, bool upper, int64_t n, int64_t nrhs, const double *T, int64_t lda, double *B,
              int64_t ldb)
{
    const int NB = 64;
    dim3 g1((unsigned)((nrhs + 255) / 256));
    if (!upper) {
        for (int64_t b0 = 0; b0 < n; b0 += NB) {  // L y = b
            int nb = (int)std::min<int64_t>(NB, n - b0);
            hipLaunchKernelGGL(k_trsm_blk, g1, dim3(256), 0, s, b0, nb, T, lda, B, ldb, nrhs, 0);
            int64_t rest = n - b0 - nb;
            if (rest > 0)
                gemm_f64(s, false, false, rest, nrhs, nb, -1.0, T + (b0 + nb) * lda + b0, lda,
                         B + b0 * ldb, ldb, 1.0, B + (b0 + nb) * ldb, ldb);
        }
    } else {
        for (int64_t b0 = ((n - 1) / NB) * NB; b0 >= 0; b0 -= NB) {  // U x = y
            int nb = (int)std::min<int64_t>(NB, n - b0);
            hipLaunchKernelGGL(k_trsm_blk, g1, dim3(256), 0, s, b0, nb, T, lda, B, ldb, nrhs, 1);
            if (b0 > 0)
                gemm_f64(s, false, false, b0, nrhs, nb, -1.0, T + b0, lda, B + b0 * ldb, ldb, 1.0, B, ldb);
        }
    }
}

void getrs_f64(hipStream_t s, bool trans, int64_t n, int64_t nrhs, const double *LU, int64_t lda,
               const int32_t *ipiv, double *B, int64_t ldb)
{
    const int NB = 64;
    dim3 g1((unsigned)((nrhs + 255) / 256));
    if (!trans) {
        hipLaunchKernelGGL(k_rowswap, g1, dim3(256), 0, s, n, nrhs, B, ldb, ipiv, 0);
        trsm_f64(s, false, n, nrhs, LU, lda, B, ldb);
        trsm_f64(s, true, n, nrhs, LU, lda, B, ldb);
    } else {
        for (int64_t b0 = 0; b0 < n; b0 += NB) {  // U^T z = b (lower)
            int nb = (int)std::min<int64_t>(NB, n - b0);
            hipLaunchKernelGGL(k_trsm_blk, g1, dim3(256), 0, s, b0, nb, LU, lda, B, ldb, nrhs, 2);
            int64_t rest = n - b0 - nb;
            if (rest > 0)  // B[rest] -= (U[b0:b0+nb, b0+nb:])^T z
                gemm_f64(s, true, false, rest, nrhs, nb, -1.0, LU + b0 * lda + b0 + nb, lda,
                         B + b0 * ldb, ldb, 1.0, B + (b0 + nb) * ldb, ldb);
        }
        for (int64_t b0 = ((n - 1) / NB) * NB; b0 >= 0; b0 -= NB) {  // L^T w = z (upper, unit)
            int nb = (int)std::min<int64_t>(NB, n - b0);
            hipLaunchKernelGGL(k_trsm_blk, g1, dim3(256), 0, s, b0, nb, LU, lda, B, ldb, nrhs, 3);
            if (b0 > 0)  // B[0:b0] -= (L[b0:b0+nb, 0:b0])^T w
                gemm_f64(s, true, false, b0, nrhs, nb, -1.0, LU + b0 * lda, lda, B + b0 * ldb, ldb,
                         1.0, B, ldb);
        }
        hipLaunchKernelGGL(k_rowswap, g1, dim3(256), 0, s, n, nrhs, B, ldb, ipiv, 1);
    }
}

__global__ void k_count_nonzero(int64_t n, const double *x, unsigned long long *count)
{
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += x[i] != 0.0;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}
void count_nonzero(hipStream_t s, int64_t n, const double *x, unsigned long long *count)
{
    hipLaunchKernelGGL(k_count_nonzero, dim3(1024), dim3(256), 0, s, n, x, count);
}

}  // namespace qhp
