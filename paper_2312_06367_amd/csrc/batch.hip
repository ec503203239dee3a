// Grouped per-step kernels for a batch of independent scatterers (uneven
// sizes) marched together: every kernel covers all scatterers through a
// descriptor table, reads the per-scatterer step and ring head from device
// memory, and can therefore be captured once in a HIP graph and replayed
// every step.  The products are of the multi-right-hand-side streaming GEMV
// form of the single-scatterer history kernel (Sec. IV-B: b_i = r_i -
// sum_k T_k y_{i-k}; y_i = T_0^{-1} b_i; eq. post_processing).
#include "batch.h"

#include <algorithm>

namespace qhp {

static unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T>
struct GSt;
template <>
struct GSt<double> {
    static constexpr int N = 2;
    typedef double v_t __attribute__((ext_vector_type(2)));
};
template <>
struct GSt<float> {
    static constexpr int N = 4;
    typedef float v_t __attribute__((ext_vector_type(4)));
};

// Work-queue GEMV over all groups.  A tile is (group, block of 16 rows, lag
// split); tiles are taken from a device counter so that large scatterers do
// not leave CUs idle.  partial[split][row][rhs] += over the split's lags of
// A_k[row] . x_{slot(k)}[.][rhs].
template <typename T, typename Y, typename A, int NR>
__global__ __launch_bounds__(256) void k_grouped_gemv(const GDesc *__restrict__ gd, int ngroups, int64_t total_tiles,
                                                      unsigned long long *counter)
{
    constexpr int VN = GSt<T>::N;
    constexpr int RPW = 4;
    typedef typename GSt<T>::v_t V;
    __shared__ int64_t s_tile;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (;;) {
        if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(counter, 1ull);
        __syncthreads();
        const int64_t tile = s_tile;
        __syncthreads();
        if (tile >= total_tiles) return;
        int g = 0;
        while (g + 1 < ngroups && gd[g + 1].tile0 <= tile) ++g;
        const GDesc d = gd[g];
        const int64_t local = tile - d.tile0;
        const int64_t rb = local % d.rowblocks, sp = local / d.rowblocks;
        const int64_t row0 = rb * 16 + wave * RPW;
        const int64_t lps = (d.nlags + d.nsplit - 1) / d.nsplit;
        const int64_t k0 = sp * lps;
        const int64_t k1 = (k0 + lps < d.nlags) ? k0 + lps : d.nlags;
        const int64_t head = d.head ? *d.head : 0;
        A acc[RPW][NR];
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr)
#pragma unroll
            for (int b = 0; b < NR; ++b) acc[rr][b] = 0;
        for (int64_t k = k0; k < k1; ++k) {
            const Y *x = (const Y *)d.x + ((head + k) % d.n_slots) * d.x_slot_stride;
            const T *Ak = (const T *)d.A + k * d.lag_stride;
            A part[RPW][NR];
#pragma unroll
            for (int rr = 0; rr < RPW; ++rr)
#pragma unroll
                for (int b = 0; b < NR; ++b) part[rr][b] = 0;
            for (int64_t c0 = (int64_t)lane * VN; c0 < d.cols; c0 += 64 * VN) {
                A xv[VN][NR];
#pragma unroll
                for (int q = 0; q < VN; ++q)
#pragma unroll
                    for (int b = 0; b < NR; ++b)
                        xv[q][b] = (c0 + q < d.cols) ? (A)x[(c0 + q) * NR + b] : (A)0;
#pragma unroll
                for (int rr = 0; rr < RPW; ++rr) {
                    if (row0 + rr >= d.rows) continue;
                    V v = __builtin_nontemporal_load(reinterpret_cast<const V *>(Ak + (row0 + rr) * d.ld + c0));
#pragma unroll
                    for (int q = 0; q < VN; ++q) {
                        A t = (c0 + q < d.cols) ? (A)v[q] : (A)0;
#pragma unroll
                        for (int b = 0; b < NR; ++b) part[rr][b] += t * xv[q][b];
                    }
                }
            }
            const A sc = d.scales ? (A)d.scales[k] : (A)1;
#pragma unroll
            for (int rr = 0; rr < RPW; ++rr)
#pragma unroll
                for (int b = 0; b < NR; ++b) acc[rr][b] += sc * part[rr][b];
        }
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr)
#pragma unroll
            for (int b = 0; b < NR; ++b) {
                A v = acc[rr][b];
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                acc[rr][b] = v;
            }
        if (lane == 0) {
            A *out = (A *)d.partial + sp * d.rows * NR;
#pragma unroll
            for (int rr = 0; rr < RPW; ++rr)
                if (row0 + rr < d.rows)
#pragma unroll
                    for (int b = 0; b < NR; ++b) out[(row0 + rr) * NR + b] = acc[rr][b];
        }
    }
}

// Multi-right-hand-side form of the same work-queue product: a tile is
// 4 * RW rows (RW per wave); the (lag, column chunk) steps of the tile are
// walked as one sequence of chunks of 64 * VN columns.  For each chunk the x
// values of all NR right-hand sides are staged once in LDS and shared by
// every row of the tile; each lane keeps one vector of columns of each of its
// rows.  Software pipeline: while chunk t is multiplied, the lag-block
// vectors and the x values of chunk t + 1 are already in flight (registers),
// and the x values land in the other half of a double-buffered LDS area, so
// one barrier per chunk suffices.  The LDS copy is padded by 16 bytes per
// lane block so that the 16-byte reads of a lane group fall in distinct banks.
// Requires the columns [cols, ld) of every block to hold finite values (the
// library keeps them zero).
template <typename T, typename Y, typename A, int NR, int RW, int MINB = (sizeof(A) == 8 ? 2 : 3)>
__global__ __launch_bounds__(256, MINB) void k_grouped_mrhs(const GDesc *__restrict__ gd, int ngroups,
                                                      int64_t total_tiles, unsigned long long *counter)
{
    constexpr int VN = GSt<T>::N;
    constexpr int CH = 64 * VN;
    constexpr int ROWS = 4 * RW;
    constexpr int PAD = 16 / sizeof(Y);
    constexpr int LB = VN * NR + PAD;   // LDS elements per lane block of VN columns
    constexpr int XPT = CH * NR / 256;  // x elements staged per thread and chunk
    typedef typename GSt<T>::v_t V;
    __shared__ Y xs[2][64 * LB];
    __shared__ int64_t s_tile;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (;;) {
        __syncthreads();  // the previous tile's last chunk has been read
        if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(counter, 1ull);
        __syncthreads();
        const int64_t tile = s_tile;
        if (tile >= total_tiles) return;
        int g = 0;
        while (g + 1 < ngroups && gd[g + 1].tile0 <= tile) ++g;
        const GDesc d = gd[g];
        const int64_t local = tile - d.tile0;
        const int64_t rb = local % d.rowblocks, sp = local / d.rowblocks;
        const int64_t row0 = rb * ROWS + wave * RW;
        const int64_t lps = (d.nlags + d.nsplit - 1) / d.nsplit;
        const int64_t k0 = sp * lps;
        const int64_t k1 = (k0 + lps < d.nlags) ? k0 + lps : d.nlags;
        const int64_t head = d.head ? *d.head : 0;
        const int64_t nch = (d.cols + CH - 1) / CH;
        const int64_t total = (k1 > k0 ? k1 - k0 : 0) * nch;
        A acc[RW][NR];
#pragma unroll
        for (int rr = 0; rr < RW; ++rr)
#pragma unroll
            for (int b = 0; b < NR; ++b) acc[rr][b] = 0;
        V v[RW];
        Y xr[XPT];
        // x values of chunk t (lag k0 + t / nch, columns (t % nch) * CH + ...)
        auto load_x = [&](int64_t t) {
            const int64_t k = k0 + t / nch, c0 = (t % nch) * CH;
            const Y *x = (const Y *)d.x + ((head + k) % d.n_slots) * d.x_slot_stride + c0 * NR;
            const int64_t nel = (d.cols - c0 < CH ? d.cols - c0 : CH) * NR;
#pragma unroll
            for (int j = 0; j < XPT; ++j) {
                const int e = threadIdx.x + 256 * j;
                xr[j] = e < nel ? x[e] : (Y)0;
            }
        };
        // lag-block vector of row rr in chunk t (zero past the last column)
        auto load_row = [&](int64_t t, int rr) {
            const int64_t k = k0 + t / nch, c = (t % nch) * CH + (int64_t)lane * VN;
            if (c < d.cols && row0 + rr < d.rows)
                v[rr] = __builtin_nontemporal_load(
                    reinterpret_cast<const V *>((const T *)d.A + k * d.lag_stride + (row0 + rr) * d.ld + c));
            else
                v[rr] = V{};
        };
        auto stage = [&](int buf) {
#pragma unroll
            for (int j = 0; j < XPT; ++j) {
                const int e = threadIdx.x + 256 * j;
                const int cc = e / NR, b = e % NR;
                xs[buf][(cc / VN) * LB + (cc % VN) * NR + b] = xr[j];
            }
        };
        if (total > 0) {
            load_x(0);
#pragma unroll
            for (int rr = 0; rr < RW; ++rr) load_row(0, rr);
            stage(0);
        }
        __syncthreads();
        for (int64_t t = 0; t < total; ++t) {
            const int buf = (int)(t & 1);
            const bool more = t + 1 < total;
            if (more) load_x(t + 1);
            A xv[VN][NR];
#pragma unroll
            for (int q = 0; q < VN; ++q)
#pragma unroll
                for (int b = 0; b < NR; ++b) xv[q][b] = (A)xs[buf][lane * LB + q * NR + b];
            // columns past the last one hold zeros in both operands (zero padding
            // of the blocks, zero-filled x), so no masking is needed here
#pragma unroll
            for (int rr = 0; rr < RW; ++rr) {
#pragma unroll
                for (int q = 0; q < VN; ++q) {
                    const A tv = (A)v[rr][q];
#pragma unroll
                    for (int b = 0; b < NR; ++b) acc[rr][b] += tv * xv[q][b];
                }
                if (more) load_row(t + 1, rr);  // the register is free again
            }
            if (more) stage(buf ^ 1);
            __syncthreads();
        }
#pragma unroll
        for (int rr = 0; rr < RW; ++rr)
#pragma unroll
            for (int b = 0; b < NR; ++b) {
                A x = acc[rr][b];
                for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
                acc[rr][b] = x;
            }
        if (lane == 0) {
            A *out = (A *)d.partial + sp * d.rows * NR;
#pragma unroll
            for (int rr = 0; rr < RW; ++rr)
                if (row0 + rr < d.rows)
#pragma unroll
                    for (int b = 0; b < NR; ++b) out[(row0 + rr) * NR + b] = acc[rr][b];
        }
    }
}

// Multi-right-hand-side form with FP32 blocks on a transposed ring ([nrhs]
// [x_ld] per slot, Y = float for FP32 sums, double for FP64 y and sums),
// staged in registers: the 64 lanes of a wave are CG column lanes times
// 64 / CG row groups of RW rows.  For each chunk of 4 CG columns a lane loads
// one 16-byte vector of each of its rows and the four matching entries of
// each right-hand side, fully coalesced, with no LDS and no barrier in the
// streaming loop; the 64 / CG row groups of a wave ask for the same entries
// of the right-hand sides, so fewer distinct cache lines are read per load
// when CG < 64.  Columns past the last one are zero in both operands.
template <typename Y, typename A, int NR, int RW, int CG>
__global__ __launch_bounds__(256) void k_grouped_mrhs_t(const GDesc *__restrict__ gd, int ngroups,
                                                        int64_t total_tiles, unsigned long long *counter)
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    typedef Y y4 __attribute__((ext_vector_type(4)));
    constexpr int ROWS_W = (64 / CG) * RW, ROWS = 4 * ROWS_W;
    __shared__ int64_t s_tile;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cg = lane % CG, rg = lane / CG;
    for (;;) {
        if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(counter, 1ull);
        __syncthreads();
        const int64_t tile = s_tile;
        __syncthreads();
        if (tile >= total_tiles) return;
        int g = 0;
        while (g + 1 < ngroups && gd[g + 1].tile0 <= tile) ++g;
        const GDesc d = gd[g];
        const int64_t local = tile - d.tile0;
        const int64_t rb = local % d.rowblocks, sp = local / d.rowblocks;
        const int64_t row0 = rb * ROWS + wave * ROWS_W + rg * RW;
        const int64_t lps = (d.nlags + d.nsplit - 1) / d.nsplit;
        const int64_t k0 = sp * lps;
        const int64_t k1 = (k0 + lps < d.nlags) ? k0 + lps : d.nlags;
        const int64_t head = d.head ? *d.head : 0;
        A acc[RW][NR];
#pragma unroll
        for (int rr = 0; rr < RW; ++rr)
#pragma unroll
            for (int b = 0; b < NR; ++b) acc[rr][b] = 0;
        for (int64_t k = k0; k < k1; ++k) {
            const Y *x = (const Y *)d.x + ((head + k) % d.n_slots) * d.x_slot_stride;
            const float *Ak = (const float *)d.A + k * d.lag_stride;
            for (int64_t c = 4 * (int64_t)cg; c < d.cols; c += 4 * CG) {
                y4 xv[NR];
                f4 v[RW];
#pragma unroll
                for (int b = 0; b < NR; ++b) xv[b] = *reinterpret_cast<const y4 *>(x + b * d.x_ld + c);
#pragma unroll
                for (int rr = 0; rr < RW; ++rr)
                    v[rr] = row0 + rr < d.rows
                                ? __builtin_nontemporal_load(reinterpret_cast<const f4 *>(Ak + (row0 + rr) * d.ld + c))
                                : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int rr = 0; rr < RW; ++rr)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int b = 0; b < NR; ++b) acc[rr][b] += (A)v[rr][q] * (A)xv[b][q];
            }
        }
#pragma unroll
        for (int rr = 0; rr < RW; ++rr)
#pragma unroll
            for (int b = 0; b < NR; ++b) {
                A x = acc[rr][b];
                for (int off = CG / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
                acc[rr][b] = x;
            }
        if (cg == 0) {
            A *out = (A *)d.partial + sp * d.rows * NR;
#pragma unroll
            for (int rr = 0; rr < RW; ++rr)
                if (row0 + rr < d.rows)
#pragma unroll
                    for (int b = 0; b < NR; ++b) out[(row0 + rr) * NR + b] = acc[rr][b];
        }
    }
}

// The same product staged in LDS.  A tile's steps are (lag, chunk of 64
// columns); each step's block rows (4 rows x 256 bytes per 1 KB piece) and
// right-hand-side entries are copied straight from memory into one of NB LDS
// buffers (global_load_lds, 16 bytes a lane; the block rows with the
// nontemporal cache policy, as they are read once), NB - 1 steps ahead of the
// arithmetic, so a wave keeps the copies in flight without holding them in
// registers.  Each wave waits only for its own copies of the next step
// (vmcnt counts them exactly: no other vector memory access is issued in the
// loop), then one barrier makes every wave's copies visible.  Lanes are 16
// column lanes times 4 row groups of RW rows; the 4 row groups read the same
// right-hand-side entries (an LDS broadcast).  Columns past the last one are
// zero in both operands; rows past the last one are clamped in the copies
// and never written.  One work-group per tile (no work queue: the tiles are
// in the queue's order, biggest scatterer first, and the dispatcher starts
// them in that order), so that no copy of one tile is pending in the next.
template <typename Y, int NR, int RW, int NB, int MINW>
__global__ __launch_bounds__(256, MINW) void k_grouped_mrhs_d(const GDesc *__restrict__ gd, int ngroups,
                                                              int64_t total_tiles)
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    typedef int i4 __attribute__((ext_vector_type(4)));
    constexpr int CG = 16, ROWS_W = 4 * RW, ROWS = 4 * ROWS_W;
    constexpr int AP = ROWS / 4;                                   // block pieces of a step
    constexpr int YP = (NR * 64 * (int)sizeof(Y) + 1023) / 1024;  // right-hand-side pieces
    constexpr int PIECES = (AP + YP + 3) / 4 * 4, PW = PIECES / 4, PF = NB - 1;
    // vmcnt(PW (PF - 1)) with the other counters left alone (gfx9 encoding)
    constexpr int WAIT_INFLIGHT = ((PW * (PF - 1)) & 15) | (7 << 4) | (15 << 8) | (((PW * (PF - 1)) >> 4) << 14);
    static_assert(NB >= 2 && PW * (PF - 1) < 64, "steps in flight");
    __shared__ i4 S[NB][PIECES * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cg = lane % CG, rg = lane / CG;
    {
        const int64_t tile = blockIdx.x;
        if (tile >= total_tiles) return;
        int g = 0;
        while (g + 1 < ngroups && gd[g + 1].tile0 <= tile) ++g;
        const GDesc d = gd[g];
        const int64_t local = tile - d.tile0;
        const int64_t rb = local % d.rowblocks, sp = local / d.rowblocks;
        const int64_t trow0 = rb * ROWS;
        const int64_t lps = (d.nlags + d.nsplit - 1) / d.nsplit;
        const int64_t k0 = sp * lps;
        const int64_t k1 = (k0 + lps < d.nlags) ? k0 + lps : d.nlags;
        const int64_t head = d.head ? *d.head : 0;
        const int64_t nch = (d.cols + 63) / 64;  // ld is a multiple of 64
        const int64_t total = (k1 > k0 ? k1 - k0 : 0) * nch;
        Y acc[RW][NR];
#pragma unroll
        for (int rr = 0; rr < RW; ++rr)
#pragma unroll
            for (int b = 0; b < NR; ++b) acc[rr][b] = 0;
        if (total > 0) {
            int64_t lk = k0, lc = 0;  // copy cursor; past the end it repeats the last step
            auto load = [&](int buf) {
                const bool in = lk < k1;
                const int64_t k = in ? lk : k1 - 1, c0 = 64 * (in ? lc : nch - 1);
                const float *Ak = (const float *)d.A + k * d.lag_stride;
                const Y *xs = (const Y *)d.x + ((head + k) % d.n_slots) * d.x_slot_stride;
#pragma unroll
                for (int q = 0; q < PW; ++q) {
                    const int pc = wave + 4 * q;
                    if (pc < AP) {  // block rows: read once per step, so nontemporal (cache policy nt)
                        int64_t row = trow0 + 4 * pc + (lane >> 4);
                        row = row < d.rows ? row : d.rows - 1;
                        __builtin_amdgcn_global_load_lds((const void *)(Ak + row * d.ld + c0 + 4 * (lane & 15)),
                                                         (__attribute__((address_space(3))) void *)(&S[buf][pc * 64]),
                                                         16, 0, 2);
                    } else {  // right-hand sides [b][64 columns], re-read by every row block; padding
                              // pieces repeat the first
                        const int off = (pc < AP + YP ? pc - AP : 0) * 1024 + lane * 16;
                        int b = off / (64 * (int)sizeof(Y));
                        const int col = (off % (64 * (int)sizeof(Y))) / (int)sizeof(Y);
                        b = b < NR ? b : NR - 1;
                        __builtin_amdgcn_global_load_lds((const void *)(xs + b * d.x_ld + c0 + col),
                                                         (__attribute__((address_space(3))) void *)(&S[buf][pc * 64]),
                                                         16, 0, 0);
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
            for (int64_t t0 = 0; t0 < total; t0 += NB) {
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    if (t0 + u >= total) break;
                    // step t + PF into the buffer read one step ago (every wave is past it)
                    load((u + PF) % NB);
                    const float *Sa = reinterpret_cast<const float *>(&S[u][0]);
                    const Y *Sy = reinterpret_cast<const Y *>(&S[u][AP * 64]);
                    f4 va[RW];
#pragma unroll
                    for (int rr = 0; rr < RW; ++rr)
                        va[rr] = *reinterpret_cast<const f4 *>(Sa + (wave * ROWS_W + rg * RW + rr) * 64 + 4 * cg);
#pragma unroll
                    for (int b = 0; b < NR; ++b) {
                        Y yv[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) yv[q] = Sy[b * 64 + 4 * cg + q];
#pragma unroll
                        for (int rr = 0; rr < RW; ++rr)
#pragma unroll
                            for (int q = 0; q < 4; ++q) acc[rr][b] += (Y)va[rr][q] * yv[q];
                    }
                    // this wave's copies of step t + 1 are in; then every wave's are
                    __builtin_amdgcn_s_waitcnt(WAIT_INFLIGHT);
                    __builtin_amdgcn_s_barrier();
                }
            }
            // the copies issued past the last step land before the wave ends: vmcnt(0)
            __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));
        }
#pragma unroll
        for (int rr = 0; rr < RW; ++rr)
#pragma unroll
            for (int b = 0; b < NR; ++b) {
                Y x = acc[rr][b];
                for (int off = CG / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
                acc[rr][b] = x;
            }
        if (cg == 0) {
            const int64_t row0 = trow0 + wave * ROWS_W + rg * RW;
            Y *out = (Y *)d.partial + sp * d.rows * NR;
#pragma unroll
            for (int rr = 0; rr < RW; ++rr)
                if (row0 + rr < d.rows)
#pragma unroll
                    for (int b = 0; b < NR; ++b) out[(row0 + rr) * NR + b] = acc[rr][b];
        }
    }
}

template <typename T>
__global__ void k_ring_transpose(int64_t n_slots, int64_t ld, int64_t nrhs, const T *in, T *out)
{
    const int64_t n = n_slots * ld * nrhs;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = idx / (ld * nrhs), rem = idx % (ld * nrhs), i = rem / nrhs, b = rem % nrhs;
        out[(s * nrhs + b) * ld + i] = in[idx];
    }
}
// y [ne][nrhs] -> one slot of a transposed ring, dst[b][i] (row stride ldt);
// entries i >= ne of the slot are left as they are (zero)
__global__ void k_store_transposed(int64_t n, int64_t nrhs, int64_t ldt, const double *y, double *dst)
{
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x)
        dst[(idx % nrhs) * ldt + idx / nrhs] = y[idx];
}
void launch_store_transposed(hipStream_t s, int64_t ne, int64_t nrhs, int64_t ldt, const double *y, double *dst)
{
    const int64_t n = ne * nrhs;
    hipLaunchKernelGGL(k_store_transposed, dim3((unsigned)std::min<int64_t>(nblk(n, 256), 1024)), dim3(256), 0, s, n,
                       nrhs, ldt, y, dst);
}
__global__ void k_set_i64(int64_t *p, int64_t v) { *p = v; }
void launch_set_i64(hipStream_t s, int64_t *p, int64_t v) { hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, p, v); }
__global__ void k_partial_finish_f64(int64_t n, int64_t nsplit, const double *partial, const double *r, double *b)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int64_t q = 0; q < nsplit; ++q) acc += partial[q * n + i];
    b[i] = r[i] - acc;
}
void launch_partial_finish_f64(hipStream_t s, int64_t n, int64_t nsplit, const double *partial, const double *r,
                               double *b)
{
    hipLaunchKernelGGL(k_partial_finish_f64, dim3(nblk(n, 256)), dim3(256), 0, s, n, nsplit, partial, r, b);
}
void launch_ring_transpose(hipStream_t s, int64_t n_slots, int64_t ld, int64_t nrhs, const float *in, float *out)
{
    hipLaunchKernelGGL(k_ring_transpose<float>, dim3(1024), dim3(256), 0, s, n_slots, ld, nrhs, in, out);
}
void launch_ring_transpose(hipStream_t s, int64_t n_slots, int64_t ld, int64_t nrhs, const double *in, double *out)
{
    hipLaunchKernelGGL(k_ring_transpose<double>, dim3(1024), dim3(256), 0, s, n_slots, ld, nrhs, in, out);
}

// tile shapes of the transposed-ring kernels that the batch's autotuner
// chooses from (FP32 sums; FP64 y and sums), the default first.  form 0:
// registers, 64 column lanes; 1: registers, 16 column lanes x 4 row groups;
// 2: LDS-staged (nb buffers, minw work-groups per CU)
struct TransVariant {
    int form, rw, nb, minw;
};
static const TransVariant kTransF32[] = {{1, 16, 0, 0}, {1, 8, 0, 0}, {0, 16, 0, 0},
                                         {0, 8, 0, 0},  {2, 8, 2, 2}, {2, 4, 3, 2}};
static const TransVariant kTransF32A[] = {{2, 4, 3, 2}, {2, 4, 4, 1}, {2, 8, 3, 1},
                                          {1, 8, 0, 0}, {0, 4, 0, 0}, {0, 8, 0, 0}};
constexpr int kNumTrans = 6;
static_assert(sizeof(kTransF32) / sizeof(kTransF32[0]) == kNumTrans, "variant table");
static_assert(sizeof(kTransF32A) / sizeof(kTransF32A[0]) == kNumTrans, "variant table");

// rows per wave of the multi-right-hand-side kernel: as many as keep the
// accumulators, the in-flight block vectors and the staged x of one lane
// within the register budget of three waves per SIMD
constexpr int mrhs_rw(int kind, int nrhs) { return (kind == GK_F32 && nrhs <= 2) ? 8 : 4; }

bool grouped_ring_transposed(int kind, int nrhs) { return (kind == GK_F32 || kind == GK_F32A) && nrhs >= 2; }

int grouped_hist_variants(int kind, int nrhs, bool transposed)
{
    return (transposed && nrhs >= 2 && kind != GK_F64) ? kNumTrans : 1;
}

static const TransVariant &trans_variant(int kind, int variant)
{
    if (variant < 0 || variant >= kNumTrans) variant = 0;
    return kind == GK_F32 ? kTransF32[variant] : kTransF32A[variant];
}

// rows of one work tile (4 waves): variant 0 is the default shape
int64_t grouped_rows_per_tile(int kind, int nrhs, bool transposed, int variant)
{
    if (nrhs == 1) return 16;
    if (transposed && (kind == GK_F32 || kind == GK_F32A)) {
        const TransVariant &t = trans_variant(kind, variant);
        return t.form == 0 ? 4 * t.rw : 16 * t.rw;
    }
    return 4 * mrhs_rw(kind, nrhs);
}

const char *grouped_variant_name(int kind, int nrhs, bool transposed, int variant)
{
    if (!(transposed && nrhs >= 2 && (kind == GK_F32 || kind == GK_F32A))) return "plain";
    static const char *names[2][kNumTrans] = {
        {"registers, 16 column lanes, 16 rows", "registers, 16 column lanes, 8 rows",
         "registers, 64 column lanes, 16 rows", "registers, 64 column lanes, 8 rows",
         "LDS-staged, 8 rows, 2 buffers, 2 groups per CU", "LDS-staged, 4 rows, 3 buffers, 2 groups per CU"},
        {"LDS-staged, 4 rows, 3 buffers, 2 groups per CU", "LDS-staged, 4 rows, 4 buffers",
         "LDS-staged, 8 rows, 3 buffers", "registers, 16 column lanes, 8 rows", "registers, 64 column lanes, 4 rows",
         "registers, 64 column lanes, 8 rows"}};
    if (variant < 0 || variant >= kNumTrans) variant = 0;
    return names[kind == GK_F32 ? 0 : 1][variant];
}

__global__ void k_reset_counter(unsigned long long *c) { *c = 0ull; }

// out[g][row][rhs] = sign_r * r_g[step][row][rhs] - sum_s partial_g[s][row][rhs]
// (r is skipped when null): the history finish (sign_r = 1) and the solve
// accumulation (r null, result negated back with sign -1).
template <typename A>
__global__ void k_grouped_finish(const GFin *__restrict__ gf, int ngroups, int64_t max_n, int negate)
{
    const int g = blockIdx.y;
    if (g >= ngroups) return;
    const GFin f = gf[g];
    const int64_t n = f.n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int64_t q = 0; q < f.nsplit; ++q) s += (double)((const A *)f.partial)[q * n + i];
        double v = negate ? s : -s;
        if (f.r) v += f.r[(*f.step) * n + i];
        f.out[i] = v;
    }
    (void)max_n;
}

// store y_i into the ring (FP64 master, optional FP32 shadow) at the new head
// slot (head - 1 mod K), optional history copy, and the non-finite check
__global__ void k_grouped_store(const GStore *__restrict__ gs, int ngroups)
{
    const int g = blockIdx.y;
    if (g >= ngroups) return;
    const GStore d = gs[g];
    const int64_t n = d.n;
    const int64_t slot = (*d.head - 1 + d.n_slots) % d.n_slots;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double v = d.y[i];
        if (!isfinite(v)) atomicExch(d.err, 2);
        d.ring64[slot * d.slot_stride + i] = v;
        if (d.ring32) d.ring32[slot * d.slot_stride + i] = (float)v;
        if (d.ring32t) d.ring32t[(slot * d.nrhs + i % d.nrhs) * d.ldt + i / d.nrhs] = (float)v;
        if (d.ring64t) d.ring64t[(slot * d.nrhs + i % d.nrhs) * d.ldt + i / d.nrhs] = v;
    }
}

// post-processing part a: s_c = sum_a sign w[edge], w = (1/dtn - 1) y_i - y_{i-1}/dtn
__global__ void k_grouped_post_a(const GPost *__restrict__ gp, int ngroups)
{
    const int g = blockIdx.y;
    if (g >= ngroups) return;
    const GPost d = gp[g];
    const int64_t n = d.nc * d.nrhs;
    const int64_t step = *d.step;  // steps done before this one
    const int64_t slot_new = (*d.head - 1 + d.n_slots) % d.n_slots;
    const double *y = d.ring64 + slot_new * d.slot_stride;
    const double *yp = step > 0 ? d.ring64 + (*d.head) * d.slot_stride : nullptr;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t c = idx / d.nrhs, b = idx % d.nrhs;
        double acc = 0.0;
        for (int a = 0; a < 3; ++a) {
            int64_t m = d.tri_edge[3 * c + a];
            double w = (1.0 / d.dtn - 1.0) * y[m * d.nrhs + b] - (yp ? yp[m * d.nrhs + b] : 0.0) / d.dtn;
            acc += d.tri_sign[3 * c + a] * w;
        }
        d.sv[idx] = acc;
    }
}
// part b: j = y + Sigma z into j_hist[step] (if any); then advance step and head
__global__ void k_grouped_post_b(const GPost *__restrict__ gp, int ngroups)
{
    const int g = blockIdx.y;
    if (g >= ngroups) return;
    const GPost d = gp[g];
    const int64_t n = d.ne * d.nrhs;
    const int64_t step = *d.step;
    const int64_t slot_new = (*d.head - 1 + d.n_slots) % d.n_slots;
    const double *y = d.ring64 + slot_new * d.slot_stride;
    if (!d.jhist) return;
    double *j = d.jhist + step * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t m = idx / d.nrhs, b = idx % d.nrhs;
        j[idx] = y[idx] + d.z[d.cells[2 * m] * d.nrhs + b] - d.z[d.cells[2 * m + 1] * d.nrhs + b];
    }
}
__global__ void k_grouped_advance(int64_t *steps, int64_t *heads, const int64_t *nslots, int ngroups)
{
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngroups) return;
    steps[g] += 1;
    heads[g] = (heads[g] - 1 + nslots[g]) % nslots[g];
}

void launch_grouped_gemv(hipStream_t s, int kind, int nrhs, const GDesc *gd, int ngroups, int64_t total_tiles,
                         unsigned long long *counter, bool transposed, int variant)
{
    if (variant < 0 || variant >= grouped_hist_variants(kind, nrhs, transposed)) variant = 0;
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, counter);
    unsigned grid = (unsigned)(total_tiles < 4096 ? total_tiles : 4096);
    if (grid == 0) return;
#define QHP_G1(T, Y, A) \
    hipLaunchKernelGGL((k_grouped_gemv<T, Y, A, 1>), dim3(grid), dim3(256), 0, s, gd, ngroups, total_tiles, counter)
#define QHP_GM(T, Y, A, NR, RW)                                                                                 \
    hipLaunchKernelGGL((k_grouped_mrhs<T, Y, A, NR, RW>), dim3(grid), dim3(256), 0, s, gd, ngroups, total_tiles, \
                       counter)
#define QHP_GN(T, Y, A, K)                                 \
    switch (nrhs) {                                        \
    case 1: QHP_G1(T, Y, A); break;                        \
    case 2: QHP_GM(T, Y, A, 2, mrhs_rw(K, 2)); break;      \
    case 4: QHP_GM(T, Y, A, 4, mrhs_rw(K, 4)); break;      \
    default: QHP_GM(T, Y, A, 8, mrhs_rw(K, 8)); break;     \
    }
#define QHP_GTR(Y, NR, RW, CG)                                                                              \
    hipLaunchKernelGGL((k_grouped_mrhs_t<Y, Y, NR, RW, CG>), dim3(grid), dim3(256), 0, s, gd, ngroups, total_tiles, \
                       counter)
#define QHP_GTD(Y, NR, RW, NB, MINW)                                                                        \
    hipLaunchKernelGGL((k_grouped_mrhs_d<Y, NR, RW, NB, MINW>), dim3((unsigned)total_tiles), dim3(256), 0, s, gd, \
                       ngroups, total_tiles)
#define QHP_GF(NR)                                  \
    switch (variant) {                              \
    case 1: QHP_GTR(float, NR, 8, 16); break;       \
    case 2: QHP_GTR(float, NR, 16, 64); break;      \
    case 3: QHP_GTR(float, NR, 8, 64); break;       \
    case 4: QHP_GTD(float, NR, 8, 2, 2); break;     \
    case 5: QHP_GTD(float, NR, 4, 3, 2); break;     \
    default: QHP_GTR(float, NR, 16, 16); break;     \
    }
#define QHP_GFA(NR)                                 \
    switch (variant) {                              \
    case 1: QHP_GTD(double, NR, 4, 4, 1); break;    \
    case 2: QHP_GTD(double, NR, 8, 3, 1); break;    \
    case 3: QHP_GTR(double, NR, 8, 16); break;      \
    case 4: QHP_GTR(double, NR, 4, 64); break;      \
    case 5: QHP_GTR(double, NR, 8, 64); break;      \
    default: QHP_GTD(double, NR, 4, 3, 2); break;   \
    }
    if (kind == GK_F64) { QHP_GN(double, double, double, GK_F64) }
    else if (kind == GK_F32) {
        switch (nrhs) {
        case 1: QHP_G1(float, float, float); break;
        case 2: QHP_GF(2); break;
        case 4: QHP_GF(4); break;
        default: QHP_GF(8); break;
        }
    }
    else if (transposed && nrhs >= 2) {
        switch (nrhs) {
        case 2: QHP_GFA(2); break;
        case 4: QHP_GFA(4); break;
        default: QHP_GFA(8); break;
        }
    }
    else { QHP_GN(float, double, double, GK_F32A) }
#undef QHP_GFA
#undef QHP_GF
#undef QHP_GTR
#undef QHP_GTD
#undef QHP_GN
#undef QHP_GM
#undef QHP_G1
}
void launch_grouped_finish(hipStream_t s, bool acc_double, const GFin *gf, int ngroups, int64_t max_n, int negate)
{
    dim3 grid(nblk(max_n, 256) < 1024 ? nblk(max_n, 256) : 1024, (unsigned)ngroups);
    if (acc_double) hipLaunchKernelGGL(k_grouped_finish<double>, grid, dim3(256), 0, s, gf, ngroups, max_n, negate);
    else hipLaunchKernelGGL(k_grouped_finish<float>, grid, dim3(256), 0, s, gf, ngroups, max_n, negate);
}
void launch_grouped_store(hipStream_t s, const GStore *gs, int ngroups, int64_t max_n)
{
    dim3 grid(nblk(max_n, 256) < 1024 ? nblk(max_n, 256) : 1024, (unsigned)ngroups);
    hipLaunchKernelGGL(k_grouped_store, grid, dim3(256), 0, s, gs, ngroups);
}
void launch_grouped_post(hipStream_t s, int part, const GPost *gp, int ngroups, int64_t max_n)
{
    dim3 grid(nblk(max_n, 256) < 1024 ? nblk(max_n, 256) : 1024, (unsigned)ngroups);
    if (part == 0) hipLaunchKernelGGL(k_grouped_post_a, grid, dim3(256), 0, s, gp, ngroups);
    else hipLaunchKernelGGL(k_grouped_post_b, grid, dim3(256), 0, s, gp, ngroups);
}
void launch_grouped_advance(hipStream_t s, int64_t *steps, int64_t *heads, const int64_t *nslots, int ngroups)
{
    hipLaunchKernelGGL(k_grouped_advance, dim3(nblk(ngroups, 64)), dim3(64), 0, s, steps, heads, nslots, ngroups);
}

}  // namespace qhp
