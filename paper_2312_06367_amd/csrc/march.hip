// Per-step kernels of the marching-on-in-time scheme (Sec. IV-B) on gfx950:
// the retarded history sum over the time-banded blocks T_k, the T_0 solve,
// the post-processing of eq. post_processing, and the tested incident fields.
#include "march.h"

#include "linalg.h"

#include <cstring>
#include <type_traits>

namespace qhp {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

static unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------- pulses
__device__ __forceinline__ double pulse(const qhp_wave &w, double u)
{
    if (w.pulse == 0) {
        double sig = 1.0 / (6.283185307179586476925286766559 * w.bw);
        return w.amplitude * cos(6.283185307179586476925286766559 * w.f0 * u) * exp(-u * u / (2.0 * sig * sig));
    }
    double a = 4.0 / w.w * u;
    return 4.0 * w.amplitude / (w.w * 1.7724538509055160272981674833411) * exp(-a * a);
}

__device__ __forceinline__ void radon7(int q, double &l0, double &l1, double &l2, double &w)
{
    const double s15 = 3.872983346207416885179265399782;
    const double a1 = (9.0 - 2.0 * s15) / 21.0, b1 = (6.0 + s15) / 21.0;
    const double a2 = (9.0 + 2.0 * s15) / 21.0, b2 = (6.0 - s15) / 21.0;
    const double w1 = (155.0 + s15) / 1200.0, w2 = (155.0 - s15) / 1200.0;
    switch (q) {
    case 0: l0 = l1 = l2 = 1.0 / 3.0; w = 9.0 / 40.0; break;
    case 1: l0 = a1; l1 = b1; l2 = b1; w = w1; break;
    case 2: l0 = b1; l1 = a1; l2 = b1; w = w1; break;
    case 3: l0 = b1; l1 = b1; l2 = a1; w = w1; break;
    case 4: l0 = a2; l1 = b2; l2 = b2; w = w2; break;
    case 5: l0 = b2; l1 = a2; l2 = b2; w = w2; break;
    default: l0 = b2; l1 = b2; l2 = a2; w = w2; break;
    }
}

// Local tested moments of e_in (coarse, RWG sign included) or h_in (fine,
// unsigned RT0 functions) on each triangle: out[col][tri][a], col = s*nrhs+b.
// mode 0: e on coarse triangles; mode 1: h = k x e on fine triangles.
__global__ void k_exc_local(int64_t ntri, const double *xyz, const int32_t *tri, const int32_t *sgn,
                            const qhp_wave *waves, int32_t nrhs, int64_t s0, int64_t ns, double dt,
                            int mode, double *out)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ntri * ns * nrhs) return;
    int64_t t = idx % ntri;
    int64_t col = idx / ntri;  // s_local * nrhs + b
    int b = (int)(col % nrhs);
    int64_t sl = col / nrhs;
    const qhp_wave w = waves[b];
    double P[3][3];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) P[i][k] = xyz[3 * tri[3 * t + i] + k];
    double e1[3], e2[3];
    for (int k = 0; k < 3; ++k) { e1[k] = P[1][k] - P[0][k]; e2[k] = P[2][k] - P[0][k]; }
    double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2], cz = e1[0] * e2[1] - e1[1] * e2[0];
    double A = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
    double tk = (double)(s0 + sl + 1) * dt;
    // field direction: p for e, k x p for h
    double dir[3];
    if (mode == 0) {
        for (int k = 0; k < 3; ++k) dir[k] = w.pol[k];
    } else {
        dir[0] = w.k_hat[1] * w.pol[2] - w.k_hat[2] * w.pol[1];
        dir[1] = w.k_hat[2] * w.pol[0] - w.k_hat[0] * w.pol[2];
        dir[2] = w.k_hat[0] * w.pol[1] - w.k_hat[1] * w.pol[0];
    }
    double acc[3] = {0, 0, 0};
    for (int q = 0; q < 7; ++q) {
        double l0, l1, l2, wq;
        radon7(q, l0, l1, l2, wq);
        double r[3];
        for (int k = 0; k < 3; ++k) r[k] = l0 * P[0][k] + l1 * P[1][k] + l2 * P[2][k];
        double u = tk - w.t0 - (r[0] * w.k_hat[0] + r[1] * w.k_hat[1] + r[2] * w.k_hat[2]);
        double amp = pulse(w, u) * wq * A / (2.0 * A);
        for (int a = 0; a < 3; ++a) {
            double d = 0.0;
            for (int k = 0; k < 3; ++k) d += (r[k] - P[a][k]) * dir[k];
            acc[a] += amp * d;
        }
    }
    for (int a = 0; a < 3; ++a) {
        double s = (mode == 0) ? (double)sgn[3 * t + a] : 1.0;
        out[(col * ntri + t) * 3 + a] = s * acc[a];
    }
}

// EH[col][m] = -e_m, EH[col][ne + m] = h_m
__global__ void k_exc_gather(int64_t ne, int64_t nc, int64_t nf, int64_t ncols, const int32_t *cells,
                             const int32_t *tri_edge, const double *eloc, const double *hloc,
                             const int32_t *bct_off, const int32_t *bct_entry, const int32_t *bc_tri,
                             const double *bc_flux, double *EH)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ne * ncols) return;
    int64_t m = idx % ne, col = idx / ne;
    double e = 0.0;
    for (int q = 0; q < 2; ++q) {
        int64_t c = cells[2 * m + q];
        for (int a = 0; a < 3; ++a)
            if (tri_edge[3 * c + a] == m) e += eloc[(col * nc + c) * 3 + a];
    }
    double h = 0.0;
    for (int q = bct_off[m]; q < bct_off[m + 1]; ++q) {
        int32_t en = bct_entry[q];
        int64_t t = bc_tri[en];
        const double *F = bc_flux + 3 * en;
        const double *hl = hloc + (col * nf + t) * 3;
        h += F[0] * hl[0] + F[1] * hl[1] + F[2] * hl[2];
    }
    EH[col * 2 * ne + m] = -e;
    EH[col * 2 * ne + ne + m] = h;
}

// r[s][m][b] = R[s*nrhs + b][m]
__global__ void k_permute_rhs(int64_t ne, int64_t ns, int32_t nrhs, const double *R, double *r)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ne * ns * nrhs) return;
    int b = (int)(idx % nrhs);
    int64_t m = (idx / nrhs) % ne, s = idx / (nrhs * ne);
    r[idx] = R[(s * nrhs + b) * ne + m];
}

void launch_exc_local(hipStream_t s, int64_t ntri, const double *xyz, const int32_t *tri, const int32_t *sgn,
                      const qhp_wave *waves, int32_t nrhs, int64_t s0, int64_t ns, double dt, int mode, double *out)
{
    int64_t n = ntri * ns * nrhs;
    hipLaunchKernelGGL(k_exc_local, dim3(nblk(n, 128)), dim3(128), 0, s, ntri, xyz, tri, sgn, waves, nrhs, s0, ns, dt, mode, out);
}
void launch_exc_gather(hipStream_t s, int64_t ne, int64_t nc, int64_t nf, int64_t ncols, const int32_t *cells,
                       const int32_t *tri_edge, const double *eloc, const double *hloc, const int32_t *bct_off,
                       const int32_t *bct_entry, const int32_t *bc_tri, const double *bc_flux, double *EH)
{
    hipLaunchKernelGGL(k_exc_gather, dim3(nblk(ne * ncols, 256)), dim3(256), 0, s, ne, nc, nf, ncols, cells,
                       tri_edge, eloc, hloc, bct_off, bct_entry, bc_tri, bc_flux, EH);
}
void launch_permute_rhs(hipStream_t s, int64_t ne, int64_t ns, int32_t nrhs, const double *R, double *r)
{
    hipLaunchKernelGGL(k_permute_rhs, dim3(nblk(ne * ns * nrhs, 256)), dim3(256), 0, s, ne, ns, nrhs, R, r);
}

// ------------------------------------------------------------ history sum
// Single right-hand side: partial[split][row] = sum over the split's lags of
// T_k[row] . y_{i-k}.  Block = 256 threads = 4 waves; each wave owns RPW rows.
// Each lane streams 16-byte vectors of the rows (UNR column chunks in flight),
// loading the matching y chunk once and reusing it for the wave's rows.  The
// slab stream is read with non-temporal loads (NT) so that the y vectors stay
// cached.  T = slab storage, Y = ring element, A = accumulation type.
template <typename T>
struct St;
template <>
struct St<double> {
    static constexpr int N = 2;
    typedef double v_t __attribute__((ext_vector_type(2)));
};
template <>
struct St<float> {
    static constexpr int N = 4;
    typedef float v_t __attribute__((ext_vector_type(4)));
};
template <>
struct St<uint16_t> {  // bf16 storage
    static constexpr int N = 8;
    typedef uint32_t v_t __attribute__((ext_vector_type(4)));
};

__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    uint32_t rounding = 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)((u + rounding) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h)
{
    return __uint_as_float(((uint32_t)h) << 16);
}

// MFMA operand order of a BF16 matrix with rows of ld entries: 16-row x
// 32-column tiles, each plane of a tile 512 entries = 64 lanes x 8, where lane
// r + 16 q holds row r, columns 8 q .. 8 q + 7 of the tile (the A and B
// operand pattern of v_mfma_f32_16x16x32_bf16), tiles row-tile major.
__device__ __forceinline__ int64_t packed_index(int64_t i, int64_t j, int64_t ld, int plane, int nplanes)
{
    const int64_t rt = i >> 4, r = i & 15, kc = j >> 5, w = j & 31;
    return ((rt * (ld >> 5) + kc) * nplanes + plane) * 512 + (r + 16 * (w >> 3)) * 8 + (w & 7);
}

template <typename T, bool NT>
__device__ __forceinline__ typename St<T>::v_t ldv(const T *p)
{
    typedef typename St<T>::v_t V;
    if (NT) return __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
    return *reinterpret_cast<const V *>(p);
}

template <typename A>
__device__ __forceinline__ void unpack(const St<double>::v_t &v, A *o)
{
    o[0] = (A)v[0];
    o[1] = (A)v[1];
}
template <typename A>
__device__ __forceinline__ void unpack(const St<float>::v_t &v, A *o)
{
    o[0] = (A)v[0]; o[1] = (A)v[1]; o[2] = (A)v[2]; o[3] = (A)v[3];
}
template <typename A>
__device__ __forceinline__ void unpack(const St<uint16_t>::v_t &v, A *o)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        o[2 * i] = (A)__uint_as_float(v[i] << 16);
        o[2 * i + 1] = (A)__uint_as_float(v[i] & 0xffff0000u);
    }
}

// y chunk of N elements of type Y starting at p, converted to A
template <typename Y, typename A, int N>
__device__ __forceinline__ void load_y(const Y *p, A *o)
{
    if constexpr (sizeof(Y) == 8) {
#pragma unroll
        for (int q = 0; q < N; q += 2) {
            double2 v = *reinterpret_cast<const double2 *>(p + q);
            o[q] = (A)v.x;
            o[q + 1] = (A)v.y;
        }
    } else {
#pragma unroll
        for (int q = 0; q < N; q += 4) {
            float4 v = *reinterpret_cast<const float4 *>(p + q);
            o[q] = (A)v.x; o[q + 1] = (A)v.y; o[q + 2] = (A)v.z; o[q + 3] = (A)v.w;
        }
    }
}

template <typename T, typename Y, typename A, int RPW, int UNR, bool NT>
__global__ __launch_bounds__(256) void k_hist_gemv(int64_t ne, int64_t ld, int64_t kmax, int64_t lags_per_split,
                                                   const T *__restrict__ slabs, const float *__restrict__ scales,
                                                   const Y *__restrict__ ring, int64_t n_slots, int64_t head,
                                                   A *__restrict__ partial)
{
    constexpr int VN = St<T>::N;
    constexpr int STEP = 64 * VN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * (4 * RPW) + wave * RPW;
    const int64_t k_begin = 1 + (int64_t)blockIdx.y * lags_per_split;
    int64_t k_end = k_begin + lags_per_split;
    if (k_end > kmax + 1) k_end = kmax + 1;
    A acc[RPW];
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) acc[rr] = 0;
    const bool full_rows = row0 + RPW <= ne;
    int64_t rows_here = ne - row0;
    if (rows_here > RPW) rows_here = RPW;
    for (int64_t k = k_begin; k < k_end; ++k) {
        const Y *y = ring + ((head + k - 1) % n_slots) * ld;
        const T *Tk = slabs + (k - 1) * ne * ld + row0 * ld;
        A part[RPW];
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr) part[rr] = 0;
        for (int64_t c0 = (int64_t)lane * VN; c0 < ne; c0 += STEP * UNR) {
            A yv[UNR][VN];
            bool ok[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int64_t cu = c0 + u * STEP;
                ok[u] = cu < ne;
                if (ok[u]) {
                    load_y<Y, A, VN>(y + cu, yv[u]);
                    if (cu + VN > ne) {
#pragma unroll
                        for (int q = 0; q < VN; ++q)
                            if (cu + q >= ne) yv[u][q] = 0;
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < VN; ++q) yv[u][q] = 0;
                }
            }
#pragma unroll
            for (int rr = 0; rr < RPW; ++rr) {
                if (!full_rows && rr >= rows_here) continue;
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    if (!ok[u]) continue;
                    const int64_t cu = c0 + u * STEP;
                    A tv[VN];
                    unpack<A>(ldv<T, NT>(Tk + rr * ld + cu), tv);
                    if (cu + VN > ne) {
#pragma unroll
                        for (int q = 0; q < VN; ++q)
                            if (cu + q >= ne) tv[q] = 0;
                    }
#pragma unroll
                    for (int q = 0; q < VN; ++q) part[rr] += tv[q] * yv[u][q];
                }
            }
        }
        const A sc = scales ? (A)scales[k - 1] : (A)1;
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr) acc[rr] += sc * part[rr];
    }
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
        A v = acc[rr];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[rr] = v;
    }
    if (lane == 0) {
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr)
            if (row0 + rr < ne) partial[(int64_t)blockIdx.y * ne + row0 + rr] = acc[rr];
    }
}

// The single right-hand-side history with FP32 blocks staged in LDS: a
// tile is 4 waves x RPW rows over the lags of one split; each step (lag,
// chunk of 256 columns) copies the tile's block rows (one row = one 1 KB
// piece, nontemporal) and the y chunk (cached: every row block reads it)
// straight into one of NB LDS buffers, NB - 1 steps ahead (global_load_lds,
// exact vmcnt waits, one barrier per step, one work-group per tile).  Lane l
// reads columns 4l..4l+3 of its rows and of y.  Requires ld % 256 == 0 (whole
// chunks stay inside a row); columns past ne are copied but masked in the
// products, so the padding may hold anything; rows past ne are clamped in the
// copies and never written.  Each lane sums a lag's products into a per-lag
// partial and adds that to its total once the lag is done, the order of the
// register form: with the same split count the two give identical results.
template <typename Y, typename A, int RPW, int NB, int MINW>
__global__ __launch_bounds__(256, MINW) void k_hist_gemv_d(int64_t ne, int64_t ld, int64_t kmax,
                                                           int64_t lags_per_split, const float *__restrict__ slabs,
                                                           const Y *__restrict__ ring, int64_t n_slots, int64_t head,
                                                           A *__restrict__ partial)
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    typedef int i4 __attribute__((ext_vector_type(4)));
    constexpr int AP = 4 * RPW;                          // block pieces of a step
    constexpr int YP = (256 * (int)sizeof(Y)) / 1024;    // y pieces
    constexpr int PIECES = (AP + YP + 3) / 4 * 4, PW = PIECES / 4, PF = NB - 1;
    // vmcnt(PW (PF - 1)) with the other counters left alone (gfx9 encoding)
    constexpr int WAIT_INFLIGHT = ((PW * (PF - 1)) & 15) | (7 << 4) | (15 << 8) | (((PW * (PF - 1)) >> 4) << 14);
    constexpr int WAIT_DRAINED = (7 << 4) | (15 << 8);  // vmcnt(0)
    static_assert(NB >= 2 && PW * (PF - 1) < 64 && YP >= 1, "pipeline shape");
    __shared__ i4 S[NB][PIECES * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t trow0 = (int64_t)blockIdx.x * AP;
    const int64_t k_begin = 1 + (int64_t)blockIdx.y * lags_per_split;
    const int64_t k_end = (k_begin + lags_per_split < kmax + 1) ? k_begin + lags_per_split : kmax + 1;
    const int64_t nch = (ne + 255) / 256;  // chunks of 256 columns (ld is a multiple of 256)
    const int64_t total = (k_end > k_begin ? k_end - k_begin : 0) * nch;
    A acc[RPW], part[RPW];
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) acc[rr] = part[rr] = 0;
    if (total > 0) {
        int64_t lk = k_begin, lc = 0;  // copy cursor; past the end it repeats the last step
        auto load = [&](int buf) {
            const bool in = lk < k_end;
            const int64_t k = in ? lk : k_end - 1, c0 = 256 * (in ? lc : nch - 1);
            const float *Tk = slabs + (k - 1) * ne * ld;
            const Y *y = ring + ((head + k - 1) % n_slots) * ld;
#pragma unroll
            for (int q = 0; q < PW; ++q) {
                const int pc = wave + 4 * q;
                if (pc < AP) {  // block row: read once, nontemporal
                    int64_t row = trow0 + pc;
                    row = row < ne ? row : ne - 1;
                    __builtin_amdgcn_global_load_lds((const void *)(Tk + row * ld + c0 + 4 * lane),
                                                     (__attribute__((address_space(3))) void *)(&S[buf][pc * 64]), 16,
                                                     0, 2);
                } else {  // the y chunk; padding pieces repeat its first piece
                    const int off = (pc < AP + YP ? pc - AP : 0) * 1024 + lane * 16;
                    __builtin_amdgcn_global_load_lds((const void *)(y + c0 + off / (int)sizeof(Y)),
                                                     (__attribute__((address_space(3))) void *)(&S[buf][pc * 64]), 16,
                                                     0, 0);
                }
            }
            if (++lc == nch) {
                lc = 0;
                ++lk;
            }
        };
#pragma unroll
        for (int q = 0; q < PF; ++q) load(q);
        __builtin_amdgcn_s_waitcnt(WAIT_INFLIGHT);  // step 0 is in
        __builtin_amdgcn_s_barrier();
        int64_t cc = 0;  // chunk of the step being multiplied
        for (int64_t t0 = 0; t0 < total; t0 += NB) {
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                if (t0 + u >= total) break;
                // step t + PF into the buffer read one step ago (every wave is past it)
                load((u + PF) % NB);
                const float *Sa = reinterpret_cast<const float *>(&S[u][0]);
                const Y *Sy = reinterpret_cast<const Y *>(&S[u][AP * 64]);
                const int64_t lim = ne - 256 * cc - 4 * lane;  // columns of this lane inside the matrix
                A yv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) yv[q] = q < lim ? (A)Sy[4 * lane + q] : (A)0;
#pragma unroll
                for (int rr = 0; rr < RPW; ++rr) {
                    const f4 va = *reinterpret_cast<const f4 *>(Sa + (wave * RPW + rr) * 256 + 4 * lane);
#pragma unroll
                    for (int q = 0; q < 4; ++q) part[rr] += (q < lim ? (A)va[q] : (A)0) * yv[q];
                }
                if (++cc == nch) {  // the lag is done
                    cc = 0;
#pragma unroll
                    for (int rr = 0; rr < RPW; ++rr) {
                        acc[rr] += part[rr];
                        part[rr] = 0;
                    }
                }
                // this wave's copies of step t + 1 are in; then every wave's are
                __builtin_amdgcn_s_waitcnt(WAIT_INFLIGHT);
                __builtin_amdgcn_s_barrier();
            }
        }
        // the copies issued past the last step (they repeat it) land before the wave ends
        __builtin_amdgcn_s_waitcnt(WAIT_DRAINED);
    }
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
        A v = acc[rr];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[rr] = v;
    }
    if (lane == 0) {
        const int64_t row0 = trow0 + wave * RPW;
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr)
            if (row0 + rr < ne) partial[(int64_t)blockIdx.y * ne + row0 + rr] = acc[rr];
    }
}

// b[row] = r[row] - sum_s partial[s][row]   (FP64 result)
template <typename A>
__global__ void k_hist_finish(int64_t n, int64_t nsplit, const A *partial, const double *r, double *b)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t q = 0; q < nsplit; ++q) s += (double)partial[q * n + i];
    b[i] = r[i] - s;
}

// variant table of the single right-hand-side kernel (autotuned per context):
// rows per wave, column chunks in flight, nontemporal block loads; the last
// two (unr = 0) are the LDS-staged kernel with 3 buffers (FP32 blocks without
// per-block scales and with ld % 256 == 0; otherwise variant 2 runs in their
// place)
struct GemvVariant {
    int rpw, unr, nt;
};
static const GemvVariant kGemvVariants[] = {{4, 1, 0}, {4, 2, 0}, {4, 2, 1}, {8, 1, 1}, {8, 2, 1}, {2, 4, 1},
                                             {4, 4, 1}, {2, 8, 1}, {8, 4, 1}, {4, 0, 1}, {8, 0, 1}};
constexpr int kNumGemvVariants = sizeof(kGemvVariants) / sizeof(kGemvVariants[0]);
int gemv_variant_count() { return kNumGemvVariants; }
void gemv_variant_desc(int v, int *rpw, int *unr, int *nt)
{
    *rpw = kGemvVariants[v].rpw;
    *unr = kGemvVariants[v].unr;
    *nt = kGemvVariants[v].nt;
}

template <typename T, typename Y, typename A>
static void gemv_dispatch(int v, hipStream_t s, int64_t ne, int64_t ld, int64_t kmax, int64_t lps, int nsplit,
                          const void *slabs, const float *scales, const void *ring, int64_t n_slots, int64_t head,
                          void *partial)
{
#define QHP_GEMV_CASE(IDX, R, U, N)                                                                          \
    case IDX:                                                                                                  \
        hipLaunchKernelGGL((k_hist_gemv<T, Y, A, R, U, N>), dim3(nblk(ne, 4 * R), (unsigned)nsplit), dim3(256), \
                           0, s, ne, ld, kmax, lps, (const T *)slabs, scales, (const Y *)ring, n_slots, head,    \
                           (A *)partial);                                                                      \
        break;
#define QHP_GEMV_DMA(IDX, R, MINW)                                                                                  \
    case IDX:                                                                                                      \
        if constexpr (std::is_same<T, float>::value) {                                                             \
            if (!scales && ld % 256 == 0) {                                                                        \
                hipLaunchKernelGGL((k_hist_gemv_d<Y, A, R, 3, MINW>), dim3(nblk(ne, 4 * R), (unsigned)nsplit),    \
                                   dim3(256), 0, s, ne, ld, kmax, lps, (const float *)slabs, (const Y *)ring,      \
                                   n_slots, head, (A *)partial);                                                   \
                break;                                                                                             \
            }                                                                                                      \
        }                                                                                                          \
        hipLaunchKernelGGL((k_hist_gemv<T, Y, A, 4, 2, true>), dim3(nblk(ne, 16), (unsigned)nsplit), dim3(256), 0, \
                           s, ne, ld, kmax, lps, (const T *)slabs, scales, (const Y *)ring, n_slots, head,         \
                           (A *)partial);                                                                          \
        break;
    switch (v) {
        QHP_GEMV_DMA(9, 4, 2)
        QHP_GEMV_DMA(10, 8, 1)
        QHP_GEMV_CASE(0, 4, 1, false)
        QHP_GEMV_CASE(1, 4, 2, false)
        QHP_GEMV_CASE(2, 4, 2, true)
        QHP_GEMV_CASE(3, 8, 1, true)
        QHP_GEMV_CASE(4, 8, 2, true)
        QHP_GEMV_CASE(5, 2, 4, true)
        QHP_GEMV_CASE(6, 4, 4, true)
        QHP_GEMV_CASE(7, 2, 8, true)
        default:
        QHP_GEMV_CASE(8, 8, 4, true)
    }
#undef QHP_GEMV_CASE
#undef QHP_GEMV_DMA
}

// Batched right-hand sides: C[row][rhs] partials with FP32 MFMA
// (v_mfma_f32_32x32x2f32: lane l holds A[l%32][l/32], B[l/32][l%32];
// result D[8*(r/4) + 4*(l/32) + r%4][l%32] in register r).
// Block tile 64 rows x 64 rhs, k-tile 32, 4 waves of 32x32.
template <typename T>
__global__ __launch_bounds__(256) void k_hist_gemm(int64_t ne, int64_t ld, int64_t nrhs, int64_t kmax,
                                                   int64_t lags_per_split, const T *__restrict__ slabs,
                                                   const float *__restrict__ scales,
                                                   const float *__restrict__ ring, int64_t n_slots,
                                                   int64_t head, float *__restrict__ partial)
{
    __shared__ float As[32][64 + 4];  // [kk][row]
    __shared__ float Bs[32][64 + 4];  // [kk][rhs]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.z * 64;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int64_t k_begin = 1 + (int64_t)blockIdx.y * lags_per_split;
    int64_t k_end = k_begin + lags_per_split;
    if (k_end > kmax + 1) k_end = kmax + 1;
    f16v acc;
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
    for (int64_t k = k_begin; k < k_end; ++k) {
        const float sc = scales ? scales[k - 1] : 1.f;
        const T *Tk = slabs + (k - 1) * ne * ld;
        const float *Y = ring + ((head + k - 1) % n_slots) * ld * nrhs;
        for (int64_t kk0 = 0; kk0 < ne; kk0 += 32) {
            // A tile: 64 rows x 32 cols of T_k (scaled), B tile: 32 rows x 64 rhs of y
            for (int e = tid; e < 64 * 32; e += 256) {
                int rr = e >> 5, kk = e & 31;
                int64_t gr = r0 + rr, gk = kk0 + kk;
                float v = 0.f;
                if (gr < ne && gk < ne) {
                    if constexpr (sizeof(T) == 2) v = __uint_as_float(((uint32_t)Tk[gr * ld + gk]) << 16);
                    else v = (float)Tk[gr * ld + gk];
                }
                As[kk][rr] = v * sc;
                int kb = e >> 6, cc = e & 63;
                int64_t gkb = kk0 + kb, gc = c0 + cc;
                Bs[kb][cc] = (gkb < ne && gc < nrhs) ? Y[gkb * nrhs + gc] : 0.f;
            }
            __syncthreads();
#pragma unroll
            for (int kq = 0; kq < 32; kq += 2) {
                float a = As[kq + (lane >> 5)][wr + (lane & 31)];
                float b = Bs[kq + (lane >> 5)][wc + (lane & 31)];
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
            }
            __syncthreads();
        }
    }
    float *out = partial + (int64_t)blockIdx.y * ne * nrhs;
    for (int rg = 0; rg < 16; ++rg) {
        int64_t gr = r0 + wr + 8 * (rg >> 2) + 4 * (lane >> 5) + (rg & 3);
        int64_t gc = c0 + wc + (lane & 31);
        if (gr < ne && gc < nrhs) out[gr * nrhs + gc] = acc[rg];
    }
}

// Batched history on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// sums).  y is held per ring slot as three BF16 terms hi, mid, lo (y ~ hi +
// mid + lo to 24 significant bits) stored in MFMA operand order ([nrp / 16]
// [ld / 32][3][512], see packed_index), so each 16 x 32 operand tile is one
// contiguous 1 KB piece per term.  PAIR (QHP_BF16X2): the lag block is a BF16
// pair, hi and lo planes stored in the same operand order (one coalesced
// 1 KB load per operand and wave), and each term takes the five products of
// relative weight >= 2^-16, T_hi (y_hi + y_mid + y_lo) + T_lo (y_hi + y_mid).
// Otherwise (QHP_BF16) the block is one row-major BF16 plane with a
// per-block scale and two products T (y_hi + y_mid), the accumulators being
// kept in units of the current block's scale (rescaled by the ratio at each
// lag change, by the last scale at the end).
// Work-group: 4 waves x 32 rows, 128 right-hand sides; the B tiles of each
// 32-column step are staged in double-buffered LDS (contiguous copies), A
// goes straight to registers DA steps ahead; one barrier per step.  Columns
// at or past ne are masked.
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u4_t __attribute__((ext_vector_type(4)));

// zero the BF16 entries of an 8-entry vector whose column first + j >= ne
__device__ __forceinline__ u4_t mask_cols(u4_t v, int64_t first, int64_t ne)
{
    if (first + 8 <= ne) return v;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (first + j >= ne) v[j >> 1] &= (j & 1) ? 0x0000ffffu : 0xffff0000u;
    return v;
}

template <bool PAIR>
__global__ __launch_bounds__(256, 2) void k_hist_mfma(int64_t ne, int64_t ld, int64_t nrp, int64_t nrhs, int64_t kmax,
                                                      int64_t lps, const uint16_t *__restrict__ slabs,
                                                      const float *__restrict__ scales,
                                                      const uint16_t *__restrict__ ringb, int64_t n_slots,
                                                      int64_t head, float *__restrict__ partial)
{
    constexpr int NB = 8, KS = 32;
    constexpr int NP = PAIR ? 3 : 2;         // y terms used
    constexpr int BPT = NB * NP * 64 / 256;  // 16-byte B pieces staged per thread
    constexpr int DA = 2;                    // A steps in registers
    constexpr int JB = 4;                    // n tiles per product-major group
    __shared__ u4_t Bs[2][NP][NB][64];       // [buf][term][n tile][lane]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * 128 + wave * 32;
    const int64_t jt0 = (int64_t)blockIdx.z * NB;  // first 16-wide n tile
    const int64_t k_begin = 1 + (int64_t)blockIdx.y * lps;
    const int64_t k_end = (k_begin + lps < kmax + 1) ? k_begin + lps : kmax + 1;
    const int64_t nks = (ne + KS - 1) / KS;
    const int64_t nkc = ld / KS;
    const int64_t total = (k_end > k_begin ? k_end - k_begin : 0) * nks;
    const int64_t slot_elems = (nrp / 16) * nkc * 3 * 512;
    const int64_t lag_stride = PAIR ? ((ne + 15) / 16) * 16 * ld * 2 : ne * ld;
    f4_t acc[2][NB];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[rt][j] = f4_t{0.f, 0.f, 0.f, 0.f};
    u4_t ah[DA][2], al[DA][2], breg[BPT];
    // step cursors (lag, 32-column chunk), advanced without divisions
    struct Cur {
        int64_t k, kc;
    };
    auto advance = [&](Cur &c) {
        if (++c.kc == nks) {
            c.kc = 0;
            ++c.k;
        }
    };
    auto load_a = [&](const Cur &c, u4_t *h, u4_t *l) {
        const uint16_t *Tk = slabs + (c.k - 1) * lag_stride;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            const int64_t row0 = r0 + 16 * rt;
            if (c.k < k_end && row0 < ne) {
                if constexpr (PAIR) {
                    const uint16_t *tile = Tk + (((row0 >> 4) * nkc + c.kc) * 2) * 512 + lane * 8;
                    h[rt] = __builtin_nontemporal_load(reinterpret_cast<const u4_t *>(tile));
                    l[rt] = __builtin_nontemporal_load(reinterpret_cast<const u4_t *>(tile + 512));
                } else {
                    const int64_t row = row0 + lr, col = c.kc * KS + 8 * lk;
                    h[rt] = (row < ne && col < ne)
                                ? mask_cols(__builtin_nontemporal_load(reinterpret_cast<const u4_t *>(Tk + row * ld + col)),
                                            col, ne)
                                : u4_t{0u, 0u, 0u, 0u};
                }
            } else {
                h[rt] = u4_t{0u, 0u, 0u, 0u};
                if (PAIR) l[rt] = u4_t{0u, 0u, 0u, 0u};
            }
        }
    };
    int64_t yslot_k = -1;
    const uint16_t *Y = ringb;
    auto load_b = [&](const Cur &c) {
        if (c.k != yslot_k) {  // lag change: ring slot of y_{i-k}
            yslot_k = c.k;
            Y = ringb + ((head + c.k - 1) % n_slots) * slot_elems;
        }
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            const int e = tid + 256 * q, j = e / (NP * 64), p = (e / 64) % NP, ln = e % 64;
            const int64_t jt = jt0 + j, first = c.kc * KS + 8 * (ln >> 4);
            breg[q] = (jt < nrp / 16 && first < ne)
                          ? mask_cols(*reinterpret_cast<const u4_t *>(Y + ((jt * nkc + c.kc) * 3 + p) * 512 + ln * 8),
                                      first, ne)
                          : u4_t{0u, 0u, 0u, 0u};
        }
    };
    auto store_b = [&](int buf) {
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            const int e = tid + 256 * q, j = e / (NP * 64), p = (e / 64) % NP, ln = e % 64;
            Bs[buf][p][j][ln] = breg[q];
        }
    };
    Cur ca{k_begin, 0}, cb{k_begin, 0};
    if (total > 0) {
#pragma unroll
        for (int u = 0; u < DA; ++u) {
            load_a(ca, ah[u], al[u]);
            advance(ca);
        }
        load_b(cb);
        advance(cb);
        store_b(0);
    }
    __syncthreads();
    int64_t kcur = k_begin, kccur = 0;  // step being multiplied
    for (int64_t t0 = 0; t0 < total; t0 += DA) {
#pragma unroll
        for (int u = 0; u < DA; ++u) {
            const int64_t t = t0 + u;
            if (t >= total) break;
            const int buf = (int)(t & 1);
            const bool more = t + 1 < total;
            if (more) {
                load_b(cb);
                advance(cb);
            }
            if (!PAIR && scales && t > 0 && kccur == 0) {  // lag change: keep units of the current scale
                const float ratio = scales[kcur - 2] / scales[kcur - 1];
#pragma unroll
                for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                    for (int j = 0; j < NB; ++j) acc[rt][j] *= ratio;
            }
            bf8_t a_h[2], a_l[2];
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                a_h[rt] = __builtin_bit_cast(bf8_t, ah[u][rt]);
                if (PAIR) a_l[rt] = __builtin_bit_cast(bf8_t, al[u][rt]);
            }
            // product-major order over groups of JB n tiles: 2 * JB independent
            // accumulators between two products into the same one
#pragma unroll
            for (int jb = 0; jb < NB; jb += JB) {
                bf8_t b_h[JB], b_m[JB], b_l[JB];
#pragma unroll
                for (int jj = 0; jj < JB; ++jj) {
                    b_h[jj] = __builtin_bit_cast(bf8_t, Bs[buf][0][jb + jj][lane]);
                    b_m[jj] = __builtin_bit_cast(bf8_t, Bs[buf][1][jb + jj][lane]);
                    if (PAIR) b_l[jj] = __builtin_bit_cast(bf8_t, Bs[buf][2][jb + jj][lane]);
                }
#pragma unroll
                for (int jj = 0; jj < JB; ++jj)
#pragma unroll
                    for (int rt = 0; rt < 2; ++rt)
                        acc[rt][jb + jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h[rt], b_h[jj], acc[rt][jb + jj], 0, 0, 0);
#pragma unroll
                for (int jj = 0; jj < JB; ++jj)
#pragma unroll
                    for (int rt = 0; rt < 2; ++rt)
                        acc[rt][jb + jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h[rt], b_m[jj], acc[rt][jb + jj], 0, 0, 0);
                if constexpr (PAIR) {
#pragma unroll
                    for (int jj = 0; jj < JB; ++jj)
#pragma unroll
                        for (int rt = 0; rt < 2; ++rt)
                            acc[rt][jb + jj] =
                                __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_l[rt], b_h[jj], acc[rt][jb + jj], 0, 0, 0);
#pragma unroll
                    for (int jj = 0; jj < JB; ++jj)
#pragma unroll
                        for (int rt = 0; rt < 2; ++rt)
                            acc[rt][jb + jj] =
                                __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h[rt], b_l[jj], acc[rt][jb + jj], 0, 0, 0);
#pragma unroll
                    for (int jj = 0; jj < JB; ++jj)
#pragma unroll
                        for (int rt = 0; rt < 2; ++rt)
                            acc[rt][jb + jj] =
                                __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_l[rt], b_m[jj], acc[rt][jb + jj], 0, 0, 0);
                }
            }
            load_a(ca, ah[u], al[u]);  // this stage's registers are free again
            advance(ca);
            if (more) store_b(buf ^ 1);
            if (++kccur == nks) {
                kccur = 0;
                ++kcur;
            }
            __syncthreads();
        }
    }
    const float last = (!PAIR && scales && total > 0) ? scales[k_end - 2] : 1.f;
    float *out = partial + (int64_t)blockIdx.y * ne * nrhs;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = r0 + 16 * rt + 4 * lk + r, n = 16 * (jt0 + j) + lr;
                if (row < ne && n < nrhs) out[row * nrhs + n] = last * acc[rt][j][r];
            }
}

// y [ne][nrhs] (FP64) -> the slot's three BF16 terms hi, mid, lo, each the
// rounding of what the previous ones leave, in MFMA operand order
__global__ void k_store_ybf(int64_t ne, int64_t nrhs, int64_t nrp, int64_t ld, const double *y, uint16_t *slot)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ne * nrhs) return;
    const int64_t i = idx / nrhs, n = idx % nrhs;
    double v = y[idx];
    for (int p = 0; p < 3; ++p) {
        const uint16_t h = f32_to_bf16((float)v);
        slot[packed_index(n, i, ld, p, 3)] = h;
        v -= (double)bf16_to_f32(h);
    }
    (void)nrp;
}
void launch_store_ybf(hipStream_t s, int64_t ne, int64_t nrhs, int64_t nrp, int64_t ld, const double *y,
                      uint16_t *slot)
{
    hipLaunchKernelGGL(k_store_ybf, dim3(nblk(ne * nrhs, 256)), dim3(256), 0, s, ne, nrhs, nrp, ld, y, slot);
}

int64_t ring_bf16_rows(int64_t nrhs) { return (nrhs + 15) / 16 * 16; }

int hist_splits(int64_t ne, int64_t kmax, int64_t nrhs, int32_t precision)
{
    if (precision == QHP_I8X4) return i8_hist_splits(ne, kmax, nrhs);
    if (nrhs > 1 && (precision == QHP_BF16 || precision == QHP_BF16X2)) {
        // matrix-core tiles of 128 rows x 128 right-hand sides: about eight
        // rounds of two resident work-groups per CU keep the last round short
        const int64_t tiles = ((ne + 127) / 128) * ((ring_bf16_rows(nrhs) + 127) / 128);
        int64_t want = (8 * 512 + tiles - 1) / tiles;
        return (int)(want < 1 ? 1 : (want > kmax ? kmax : want));
    }
    // enough blocks to fill 256 CUs several times over
    int64_t rowblocks = nrhs == 1 ? (ne + 15) / 16 : ((ne + 63) / 64) * ((nrhs + 63) / 64);
    int64_t want = (8 * 256 + rowblocks - 1) / rowblocks;
    if (want < 1) want = 1;
    if (want > kmax) want = kmax;
    return (int)want;
}

void launch_history(hipStream_t s, int32_t precision, int64_t ne, int64_t ld, int64_t nrhs, int64_t kmax,
                    const void *slabs, const float *scales, const void *ring, int64_t n_slots, int64_t head,
                    const double *r, double *b, void *partial, int nsplit, hipEvent_t e0, hipEvent_t e1,
                    int variant)
{
    if (kmax <= 0) {
        (void)hipMemcpyAsync(b, r, sizeof(double) * ne * nrhs, hipMemcpyDeviceToDevice, s);
        return;
    }
    int64_t lps = (kmax + nsplit - 1) / nsplit;
    if (e0) (void)hipEventRecord(e0, s);
    if (precision == QHP_I8X4) {
        launch_hist_i8(s, ne, ld, nrhs, kmax, nsplit, (const int8_t *)slabs, (const int8_t *)ring, n_slots, head,
                       (double *)partial, variant);
        if (e1) (void)hipEventRecord(e1, s);
        hipLaunchKernelGGL(k_hist_finish<double>, dim3(nblk(ne * nrhs, 256)), dim3(256), 0, s, ne * nrhs,
                           (int64_t)nsplit, (const double *)partial, r, b);
        return;
    }
    if (nrhs == 1) {
        if (variant < 0 || variant >= kNumGemvVariants) variant = 2;
        if (precision == QHP_F64)
            gemv_dispatch<double, double, double>(variant, s, ne, ld, kmax, lps, nsplit, slabs, scales, ring, n_slots,
                                                  head, partial);
        else if (precision == QHP_F32)
            gemv_dispatch<float, float, float>(variant, s, ne, ld, kmax, lps, nsplit, slabs, scales, ring, n_slots,
                                               head, partial);
        else if (precision == QHP_F32A)
            gemv_dispatch<float, double, double>(variant, s, ne, ld, kmax, lps, nsplit, slabs, scales, ring, n_slots,
                                                 head, partial);
        else
            gemv_dispatch<uint16_t, float, float>(variant, s, ne, ld, kmax, lps, nsplit, slabs, scales, ring, n_slots,
                                                  head, partial);
        if (e1) (void)hipEventRecord(e1, s);
        if (precision == QHP_F64 || precision == QHP_F32A)
            hipLaunchKernelGGL(k_hist_finish<double>, dim3(nblk(ne, 256)), dim3(256), 0, s, ne, (int64_t)nsplit,
                               (const double *)partial, r, b);
        else
            hipLaunchKernelGGL(k_hist_finish<float>, dim3(nblk(ne, 256)), dim3(256), 0, s, ne, (int64_t)nsplit,
                               (const float *)partial, r, b);
        return;
    }
    if (precision == QHP_F64) {
        // FP64 batched: one FP64 MFMA GEMM per lag into the partial buffer
        double *acc = (double *)partial;
        for (int64_t k = 1; k <= kmax; ++k) {
            const double *Tk = (const double *)slabs + (k - 1) * ne * ld;
            const double *Y = (const double *)ring + ((head + k - 1) % n_slots) * ld * nrhs;
            gemm_f64(s, false, false, ne, nrhs, ne, 1.0, Tk, ld, Y, nrhs, k == 1 ? 0.0 : 1.0, acc, nrhs);
        }
        if (e1) (void)hipEventRecord(e1, s);
        hipLaunchKernelGGL(k_hist_finish<double>, dim3(nblk(ne * nrhs, 256)), dim3(256), 0, s, ne * nrhs,
                           (int64_t)1, (const double *)acc, r, b);
        return;
    }
    if (precision == QHP_BF16 || precision == QHP_BF16X2) {
        const int64_t nrp = ring_bf16_rows(nrhs);
        dim3 gm(nblk(ne, 128), (unsigned)nsplit, nblk(nrp, 128));
        if (precision == QHP_BF16X2)
            hipLaunchKernelGGL(k_hist_mfma<true>, gm, dim3(256), 0, s, ne, ld, nrp, nrhs, kmax, lps,
                               (const uint16_t *)slabs, nullptr, (const uint16_t *)ring, n_slots, head, (float *)partial);
        else
            hipLaunchKernelGGL(k_hist_mfma<false>, gm, dim3(256), 0, s, ne, ld, nrp, nrhs, kmax, lps,
                               (const uint16_t *)slabs, scales, (const uint16_t *)ring, n_slots, head, (float *)partial);
    } else {
        dim3 grid(nblk(ne, 64), (unsigned)nsplit, nblk(nrhs, 64));
        hipLaunchKernelGGL(k_hist_gemm<float>, grid, dim3(256), 0, s, ne, ld, nrhs, kmax, lps, (const float *)slabs,
                           scales, (const float *)ring, n_slots, head, (float *)partial);
    }
    if (e1) (void)hipEventRecord(e1, s);
    hipLaunchKernelGGL(k_hist_finish<float>, dim3(nblk(ne * nrhs, 256)), dim3(256), 0, s, ne * nrhs,
                       (int64_t)nsplit, (const float *)partial, r, b);
}

// ------------------------------------------------------------------ solve
// y = Tinv b (dense FP64 inverse), one row per wave.
__global__ __launch_bounds__(256) void k_gemv_f64(int64_t n, const double *__restrict__ A,
                                                  const double *__restrict__ x, double *__restrict__ y)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const double *a = A + row * n;
    double s = 0.0;
    int64_t c0 = 0;  // columns before c0 done by the 16-byte loads
    if ((n & 1) == 0 && ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(x)) & 15) == 0) {
        // rows 16-byte aligned: chunks of 128 columns, 16 bytes a lane, four chunks in flight
        typedef double d2 __attribute__((ext_vector_type(2)));
        const int64_t nfull = n / 128;
        double s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int64_t t = 0;
        for (; t + 4 <= nfull; t += 4) {
            d2 v[4], w[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t c = (t + u) * 128 + 2 * lane;
                v[u] = *reinterpret_cast<const d2 *>(a + c);
                w[u] = *reinterpret_cast<const d2 *>(x + c);
            }
            s = fma(v[0].x, w[0].x, fma(v[0].y, w[0].y, s));
            s1 = fma(v[1].x, w[1].x, fma(v[1].y, w[1].y, s1));
            s2 = fma(v[2].x, w[2].x, fma(v[2].y, w[2].y, s2));
            s3 = fma(v[3].x, w[3].x, fma(v[3].y, w[3].y, s3));
        }
        for (; t < nfull; ++t) {
            const int64_t c = t * 128 + 2 * lane;
            const d2 v = *reinterpret_cast<const d2 *>(a + c), w = *reinterpret_cast<const d2 *>(x + c);
            s = fma(v.x, w.x, fma(v.y, w.y, s));
        }
        s += (s1 + s2) + s3;
        c0 = nfull * 128;
    }
    for (int64_t c = c0 + lane; c < n; c += 64) s += a[c] * x[c];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) y[row] = s;
}
void launch_gemv_f64(hipStream_t s, int64_t n, const double *A, const double *x, double *y)
{
    hipLaunchKernelGGL(k_gemv_f64, dim3(nblk(n, 4)), dim3(256), 0, s, n, A, x, y);
}

// --------------------------------------------------------- post-process
// y_i stored: FP64 master copy into the ring slot and FP32 shadow for the
// reduced-precision history; non-finite values raise the error flag (2), and
// so does growth (3): an entry above limit * bound, bound the largest |r_k|
// of the steps so far (limit 0: no growth check).
__global__ void k_store_y(int64_t n, const double *y, double *slot64, float *slot32, double *yhist, int *err,
                          const double *bound, double limit)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = y[i];
    if (!isfinite(v)) atomicExch(err, 2);
    else if (limit > 0.0 && fabs(v) > limit * *bound) atomicCAS(err, 0, 3);
    if (slot64) slot64[i] = v;
    if (slot32) slot32[i] = (float)v;
    if (yhist) yhist[i] = v;
}
void launch_store_y(hipStream_t s, int64_t n, const double *y, double *slot64, float *slot32, double *yhist, int *err,
                    const double *bound, double limit)
{
    hipLaunchKernelGGL(k_store_y, dim3(nblk(n, 256)), dim3(256), 0, s, n, y, slot64, slot32, yhist, err, bound,
                       bound ? limit : 0.0);
}

// out[k] = max |r[k][.]| over the per entries of each step (one work-group a step)
__global__ void k_step_absmax(int64_t per, const double *r, double *out)
{
    __shared__ double red[256];
    const double *rk = r + (int64_t)blockIdx.x * per;
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < per; i += 256) m = fmax(m, fabs(rk[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}
void launch_step_absmax(hipStream_t s, int64_t n_steps, int64_t per, const double *r, double *out)
{
    if (n_steps > 0) hipLaunchKernelGGL(k_step_absmax, dim3((unsigned)n_steps), dim3(256), 0, s, per, r, out);
}

// w = (1/dtn - 1) y_i - y_{i-1}/dtn ; s_c = sum_a sign(c,a) w[edge(c,a)]
__global__ void k_post_a(int64_t nc, int64_t nrhs, double dtn, const int32_t *tri_edge, const int32_t *tri_sign,
                         const double *y, const double *yprev, double *sv)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nc * nrhs) return;
    int64_t c = idx / nrhs, b = idx % nrhs;
    double acc = 0.0;
    for (int a = 0; a < 3; ++a) {
        int64_t m = tri_edge[3 * c + a];
        double w = (1.0 / dtn - 1.0) * y[m * nrhs + b] - (yprev ? yprev[m * nrhs + b] : 0.0) / dtn;
        acc += tri_sign[3 * c + a] * w;
    }
    sv[idx] = acc;
}
// j = y + Sigma z
__global__ void k_post_b(int64_t ne, int64_t nrhs, const int32_t *cells, const double *y, const double *z, double *j)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ne * nrhs) return;
    int64_t m = idx / nrhs, b = idx % nrhs;
    j[idx] = y[idx] + z[cells[2 * m] * nrhs + b] - z[cells[2 * m + 1] * nrhs + b];
}
void launch_post_a(hipStream_t s, int64_t nc, int64_t nrhs, double dtn, const int32_t *tri_edge,
                   const int32_t *tri_sign, const double *y, const double *yprev, double *sv)
{
    hipLaunchKernelGGL(k_post_a, dim3(nblk(nc * nrhs, 256)), dim3(256), 0, s, nc, nrhs, dtn, tri_edge, tri_sign, y,
                       yprev, sv);
}
void launch_post_b(hipStream_t s, int64_t ne, int64_t nrhs, const int32_t *cells, const double *y, const double *z,
                   double *j)
{
    hipLaunchKernelGGL(k_post_b, dim3(nblk(ne * nrhs, 256)), dim3(256), 0, s, ne, nrhs, cells, y, z, j);
}

// quantise T (FP64, [ne][ne]) into the slab store [ne][ld] with scale
// Lag-carried rounding of one lag block into its stored precision.  The value
// rounded is T_k + c_{k-1}, and c_k = (T_k + c_{k-1}) - stored_k is carried to
// the next lag (c_0 = 0), so every prefix sum over lags of the stored blocks is
// within one rounding of the exact prefix sum.  The history sum then sees the
// rounding error only through differences y_{i-k-1} - y_{i-k}.
// T: [ne] rows of stride ldt (FP64); carry: [ne][ne] FP64 or null; out: [ne][ld].
__global__ void k_quantise_slab(int64_t ne, int64_t ld, const double *T, int64_t ldt, double *carry,
                                int32_t precision, float scale, float inv_scale, void *out)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= slab_rows(precision, ne) * ld) return;
    int64_t i = idx / ld, j = idx % ld;
    if (j >= ne || i >= ne) {
        if (precision == QHP_F64) ((double *)out)[idx] = 0.0;
        else if (precision == QHP_BF16) ((uint16_t *)out)[idx] = 0;
        else if (precision == QHP_BF16X2)
            ((uint16_t *)out)[packed_index(i, j, ld, 0, 2)] = ((uint16_t *)out)[packed_index(i, j, ld, 1, 2)] = 0;
        else ((float *)out)[idx] = 0.0f;
        return;
    }
    double v = T[i * ldt + j];
    if (carry) v += carry[i * ne + j];
    double kept;
    if (precision == QHP_F64) {
        ((double *)out)[idx] = v;
        kept = v;
    } else if (precision == QHP_F32 || precision == QHP_F32A) {
        float f = (float)v;
        ((float *)out)[idx] = f;
        kept = (double)f;
    } else if (precision == QHP_BF16X2) {  // hi and lo planes, in MFMA operand order
        const uint16_t h = f32_to_bf16((float)v);
        const double hv = (double)bf16_to_f32(h);
        const uint16_t l = f32_to_bf16((float)(v - hv));
        ((uint16_t *)out)[packed_index(i, j, ld, 0, 2)] = h;
        ((uint16_t *)out)[packed_index(i, j, ld, 1, 2)] = l;
        kept = hv + (double)bf16_to_f32(l);
    } else {
        const uint16_t h = f32_to_bf16((float)v * inv_scale);
        ((uint16_t *)out)[idx] = h;
        kept = (double)bf16_to_f32(h) * (double)scale;
    }
    if (carry) carry[i * ne + j] = v - kept;
}
void launch_quantise_slab(hipStream_t s, int64_t ne, int64_t ld, const double *T, int64_t ldt, double *carry,
                          int32_t precision, float scale, void *out)
{
    hipLaunchKernelGGL(k_quantise_slab, dim3(nblk(slab_rows(precision, ne) * ld, 256)), dim3(256), 0, s, ne, ld, T,
                       ldt, carry, precision, scale, 1.0f / scale, out);
}
// FP8 E4M3 (OCP: 3 mantissa bits, exponent bias 7, subnormal quantum 2^-9,
// largest 448) rounding of y, to nearest even
__device__ __forceinline__ double round_e4m3(double y)
{
    const double ay = fabs(y);
    if (ay == 0.0) return 0.0;
    int e;
    frexp(ay, &e);  // ay = f 2^e, f in [0.5, 1): leading bit 2^(e-1)
    const double q = ldexp(1.0, (e - 1 < -6 ? -6 : e - 1) - 3);
    const double r = fmin(rint(ay / q) * q, 448.0);
    return y < 0.0 ? -r : r;
}
// per row of an [ne] x [ne] block (rows of stride ldt): the scale that maps
// max_j |T[i][j] + carry[i][j]| to 240 (1 for a zero row)
__global__ void k_fp8_rowscale(int64_t ne, const double *T, int64_t ldt, const double *carry, double *scale)
{
    const int64_t i = blockIdx.x;
    double v = 0.0;
    for (int64_t j = threadIdx.x; j < ne; j += blockDim.x) v = fmax(v, fabs(T[i * ldt + j] + carry[i * ne + j]));
    __shared__ double red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) scale[i] = red[0] > 0.0 ? red[0] / 240.0 : 1.0;
}
// FP32 words holding FP8 E4M3 values times the row scale, with the rounding
// carried to the next lag (carry = T + carry - stored); padding columns 0
__global__ void k_quantise_fp8(int64_t ne, int64_t ld, const double *T, int64_t ldt, double *carry,
                               const double *scale, float *out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ne * ld) return;
    const int64_t i = idx / ld, j = idx % ld;
    if (j >= ne) {
        out[idx] = 0.0f;
        return;
    }
    const double v = T[i * ldt + j] + carry[i * ne + j];
    const float kept = (float)(round_e4m3(v / scale[i]) * scale[i]);
    out[idx] = kept;
    carry[i * ne + j] = v - (double)kept;
}
void launch_quantise_fp8(hipStream_t s, int64_t ne, int64_t ld, const double *T, int64_t ldt, double *carry,
                         double *row_scale, float *out)
{
    hipLaunchKernelGGL(k_fp8_rowscale, dim3((unsigned)ne), dim3(256), 0, s, ne, T, ldt, carry, row_scale);
    hipLaunchKernelGGL(k_quantise_fp8, dim3(nblk(ne * ld, 256)), dim3(256), 0, s, ne, ld, T, ldt, carry, row_scale,
                       out);
}
// max |T + carry| over an [ne] x [ne] block whose rows have stride ldt
__global__ void k_absmax(int64_t ne, const double *T, int64_t ldt, const double *carry, unsigned long long *out)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    for (; idx < ne * ne; idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = idx / ne, j = idx % ne;
        double t = T[i * ldt + j] + (carry ? carry[idx] : 0.0);
        v = fmax(v, fabs(t));
    }
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(v));
}
void launch_absmax(hipStream_t s, int64_t ne, const double *T, int64_t ldt, const double *carry,
                   unsigned long long *out)
{
    hipLaunchKernelGGL(k_absmax, dim3(1024), dim3(256), 0, s, ne, T, ldt, carry, out);
}
// dequantise a stored slab into FP64 [ne][ne]
__global__ void k_load_slab(int64_t ne, int64_t ld, const void *in, int32_t precision, float scale, double *T)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ne * ne) return;
    int64_t i = idx / ne, j = idx % ne;
    int64_t o = i * ld + j;
    double v;
    if (precision == QHP_F64) v = ((const double *)in)[o];
    else if (precision == QHP_F32 || precision == QHP_F32A) v = ((const float *)in)[o];
    else if (precision == QHP_BF16X2)
        v = (double)bf16_to_f32(((const uint16_t *)in)[packed_index(i, j, ld, 0, 2)]) +
            (double)bf16_to_f32(((const uint16_t *)in)[packed_index(i, j, ld, 1, 2)]);
    else v = (double)bf16_to_f32(((const uint16_t *)in)[o]) * (double)scale;  // exact product
    T[idx] = v;
}
void launch_load_slab(hipStream_t s, int64_t ne, int64_t ld, const void *in, int32_t precision, float scale,
                      double *T)
{
    hipLaunchKernelGGL(k_load_slab, dim3(nblk(ne * ne, 256)), dim3(256), 0, s, ne, ld, in, precision, scale, T);
}

}  // namespace qhp
