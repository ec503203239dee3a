// Int8 digit storage and the batched history sum on the int8 matrix cores.
//
// The retarded history sum (Sec. IV-B) cancels strongly across lags, so it
// needs products and sums of FP64 quality even when the blocks are stored in
// four bytes: FP32 accumulation on the matrix cores, even flushed to FP64
// every few dozen columns, loses an order of magnitude more than the storage
// rounding does.  Here both operands are split into signed base-128 digits
// (an error-free splitting of a per-row / per-column fixed-point value, as
// in the integer emulations of FP64 matrix products of Ozaki et al.), the
// digit products are summed exactly in int32 over each lag, and only the
// scaling by the row and column scales and the sum over lags are rounded, in
// FP64.
#include "digits.h"

#include "../../include/qhp.h"

namespace qhp {

typedef int i4_t __attribute__((ext_vector_type(4)));

static inline unsigned nblk8(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// byte of digit a of entry (i, j) in digit planes of row stride ld: 16-row x
// 64-column tiles of 4 KB (one 1 KB matrix-core operand per digit), lane
// i % 16 + 16 (j % 64 / 16) holding bytes j % 16
__device__ __forceinline__ int64_t i8_index(int64_t i, int64_t j, int64_t ld, int a)
{
    return (((i >> 4) * (ld >> 6) + (j >> 6)) * 4 + a) * 1024 + ((i & 15) + 16 * ((j & 63) >> 4)) * 16 + (j & 15);
}

// q = rint(v * f) clamped to 127 * 2^21, then its four balanced digits
__device__ __forceinline__ int64_t fixed_q(double v, double f)
{
    double x = rint(v * f);
    const double lim = 127.0 * 2097152.0;
    x = x > lim ? lim : (x < -lim ? -lim : x);
    return (int64_t)x;
}
__device__ __forceinline__ void split4(int64_t q, int d[4])
{
    const int64_t t0 = (q + (1 << 20)) >> 21;
    q -= t0 << 21;
    const int64_t t1 = (q + (1 << 13)) >> 14;
    q -= t1 << 14;
    const int64_t t2 = (q + (1 << 6)) >> 7;
    q -= t2 << 7;
    d[0] = (int)t0;
    d[1] = (int)t1;
    d[2] = (int)t2;
    d[3] = (int)q;
}
__device__ __forceinline__ uint32_t pack4(const int *b)
{
    return (uint32_t)(b[0] & 255) | ((uint32_t)(b[1] & 255) << 8) | ((uint32_t)(b[2] & 255) << 16) |
           ((uint32_t)(b[3] & 255) << 24);
}

// ---------------------------------------------------------------- lag blocks
// row scales s_i = max_j |T(i, j) + c(i, j)| / 127 (0 for rows >= ne), one wave per row
__global__ __launch_bounds__(256) void k_i8_rowscale(int64_t ne, int64_t ld, const double *T, int64_t ldt,
                                                     const double *carry, int8_t *block)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t R = i8_rows(ne);
    if (i >= R) return;
    double m = 0.0;
    if (i < ne)
        for (int64_t j = lane; j < ne; j += 64) m = fmax(m, fabs(T[i * ldt + j] + (carry ? carry[i * ne + j] : 0.0)));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if (lane == 0) reinterpret_cast<double *>(block + R * ld * 4)[i] = m / 127.0;
}
// digits of 16 consecutive columns per thread; carry <- v - s q 2^-21
__global__ __launch_bounds__(256) void k_i8_quantise(int64_t ne, int64_t ld, const double *T, int64_t ldt,
                                                     double *carry, int8_t *block)
{
    // the carry is v minus the rounded product s q 2^-21, not a fused residual
#pragma clang fp contract(off)
    const int64_t R = i8_rows(ne), nch = ld >> 4;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= R * nch) return;
    const int64_t i = idx / nch, j0 = (idx % nch) * 16;
    uint32_t w[4][4];
    const double s = i < ne ? reinterpret_cast<const double *>(block + R * ld * 4)[i] : 0.0;
    const double f = s > 0.0 ? 2097152.0 / s : 0.0;
    for (int g = 0; g < 4; ++g) {
        int b[4][4];  // [digit][byte]
        for (int e = 0; e < 4; ++e) {
            const int64_t j = j0 + 4 * g + e;
            int d[4] = {0, 0, 0, 0};
            if (i < ne && j < ne) {
                const double v = T[i * ldt + j] + (carry ? carry[i * ne + j] : 0.0);
                int64_t q = 0;  // a row of zeros (s = 0) stores zeros exactly
                if (s > 0.0) {
                    q = fixed_q(v, f);
                    split4(q, d);
                }
                if (carry) carry[i * ne + j] = v - s * ((double)q * 0x1p-21);
            }
            for (int a = 0; a < 4; ++a) b[a][e] = d[a];
        }
        for (int a = 0; a < 4; ++a) w[a][g] = pack4(b[a]);
    }
    for (int a = 0; a < 4; ++a)
        *reinterpret_cast<i4_t *>(block + i8_index(i, j0, ld, a)) =
            i4_t{(int)w[a][0], (int)w[a][1], (int)w[a][2], (int)w[a][3]};
}
void launch_i8_quantise(hipStream_t s, int64_t ne, int64_t ld, const double *T, int64_t ldt, double *carry,
                        int8_t *block)
{
    const int64_t R = i8_rows(ne);
    hipLaunchKernelGGL(k_i8_rowscale, dim3(nblk8(R, 4)), dim3(256), 0, s, ne, ld, T, ldt, carry, block);
    hipLaunchKernelGGL(k_i8_quantise, dim3(nblk8(R * (ld >> 4), 256)), dim3(256), 0, s, ne, ld, T, ldt, carry,
                       block);
}

__global__ void k_i8_load(int64_t ne, int64_t ld, const int8_t *block, double *T)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ne * ne) return;
    const int64_t i = idx / ne, j = idx % ne;
    int64_t q = 0;
    for (int a = 0; a < 4; ++a) q = q * 128 + block[i8_index(i, j, ld, a)];
    const double s = reinterpret_cast<const double *>(block + i8_rows(ne) * ld * 4)[i];
    T[idx] = s * ((double)q * 0x1p-21);
}
void launch_i8_load(hipStream_t s, int64_t ne, int64_t ld, const int8_t *block, double *T)
{
    hipLaunchKernelGGL(k_i8_load, dim3(nblk8(ne * ne, 256)), dim3(256), 0, s, ne, ld, block, T);
}

// ---------------------------------------------------------------- history vectors
// column scales of y [ne][nrhs] (0 for padded columns), one work-group per column
__global__ __launch_bounds__(256) void k_i8_colscale(int64_t ne, int64_t nrhs, int64_t ld, const double *y,
                                                     int8_t *slot)
{
    __shared__ double red[4];
    const int64_t n = blockIdx.x, P = i8_rows(nrhs);
    double m = 0.0;
    if (n < nrhs)
        for (int64_t j = threadIdx.x; j < ne; j += 256) m = fmax(m, fabs(y[j * nrhs + n]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        reinterpret_cast<double *>(slot + P * ld * 4)[n] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3])) / 127.0;
}
// digits of 16 consecutive entries of one column per thread (threads run over columns first)
__global__ __launch_bounds__(256) void k_i8_ydigits(int64_t ne, int64_t nrhs, int64_t ld, const double *y,
                                                    int8_t *slot)
{
    const int64_t P = i8_rows(nrhs), nch = ld >> 4;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P * nch) return;
    const int64_t n = idx % P, j0 = (idx / P) * 16;
    const double s = reinterpret_cast<const double *>(slot + P * ld * 4)[n];
    const double f = s > 0.0 ? 2097152.0 / s : 0.0;
    uint32_t w[4][4];
    for (int g = 0; g < 4; ++g) {
        int b[4][4];
        for (int e = 0; e < 4; ++e) {
            const int64_t j = j0 + 4 * g + e;
            int d[4] = {0, 0, 0, 0};
            if (n < nrhs && j < ne && s > 0.0) split4(fixed_q(y[j * nrhs + n], f), d);
            for (int a = 0; a < 4; ++a) b[a][e] = d[a];
        }
        for (int a = 0; a < 4; ++a) w[a][g] = pack4(b[a]);
    }
    for (int a = 0; a < 4; ++a)
        *reinterpret_cast<i4_t *>(slot + i8_index(n, j0, ld, a)) =
            i4_t{(int)w[a][0], (int)w[a][1], (int)w[a][2], (int)w[a][3]};
}
void launch_i8_store_y(hipStream_t s, int64_t ne, int64_t nrhs, int64_t ld, const double *y, int8_t *slot)
{
    const int64_t P = i8_rows(nrhs);
    hipLaunchKernelGGL(k_i8_colscale, dim3((unsigned)P), dim3(256), 0, s, ne, nrhs, ld, y, slot);
    hipLaunchKernelGGL(k_i8_ydigits, dim3(nblk8(P * (ld >> 4), 256)), dim3(256), 0, s, ne, nrhs, ld, y, slot);
}

// ---------------------------------------------------------------- history sum
// v_mfma_i32_16x16x64_i8: lane l holds A[l % 16][16 (l / 16) + q] and
// B[16 (l / 16) + q][l % 16] (q = 0..15, one 16-byte operand each) and gets
// D[4 (l / 16) + r][l % 16] in register r, which is what the digit planes'
// 1 KB pieces hold lane by lane.
//
// Work-group: WR x WN waves; wave (wr, wn) takes RT 16-row tiles from row
// 16 RT wr and JT 16-wide right-hand-side tiles from 16 JT wn, so the
// work-group covers 16 RT WR rows x 16 JT WN right-hand sides.  A step is one
// 64-column chunk of one lag: the work-group's RT WR row tiles and JT WN
// right-hand-side tiles, four digits each (1 KB per tile and digit), go
// through registers (PF steps ahead) into double-buffered LDS, one barrier per
// step.  For each output tile, five int32 accumulators collect the digit
// products by weight 2^-7w, w = a + b <= 4 (13 products); at the end of each
// lag they are scaled by s_row s_col 2^-7w into the split's FP64 partial sums
// (the work-group owns its tile of them) and cleared.  Columns past ne hold
// zero digits.
// The 1-D grid is remapped so that each XCD (work-groups are dealt to the 8
// XCDs in turn) runs a contiguous range of (split, row tile, rhs tile) in
// that order: work-groups resident together on one XCD share the lag's y
// digits and, for several rhs tiles, the block rows in that XCD's L2.
template <int RT, int JT, int WR, int WN, int PF>
__global__ __launch_bounds__(64 * WR * WN, 1) void k_hist_i8(int64_t ne, int64_t ld, int64_t nrhs, int64_t kmax,
                                                             int64_t lps, int64_t nsplit,
                                                             const int8_t *__restrict__ slabs,
                                                             const int8_t *__restrict__ ring, int64_t n_slots,
                                                             int64_t head, double *__restrict__ partial)
{
    constexpr int NT = 64 * WR * WN;               // threads
    constexpr int TA = RT * WR, TB = JT * WN;      // tiles per step
    constexpr int QA = TA * 256 / NT, QB = TB * 256 / NT;  // 16-byte pieces per thread
    static_assert(QA * NT == TA * 256 && QB * NT == TB * 256, "pieces must divide over the threads");
    __shared__ i4_t As[2][TA * 256];  // [buf][row tile][digit][lane]
    __shared__ i4_t Bs[2][TB * 256];  // [buf][rhs tile][digit][lane]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave % WR, wn = wave / WR;
    const int64_t R = i8_rows(ne), P = i8_rows(nrhs);
    const int64_t nrt = R >> 4, nnt = P >> 4, nkc = ld >> 6;
    const int64_t blk = i8_block_bytes(ne, ld), slot_bytes = i8_slot_bytes(nrhs, ld);
    // XCD-aware order of the work-groups
    const int64_t gr = (nrt + TA - 1) / TA, gc = (nnt + TB - 1) / TB, nwg = gr * gc * nsplit;
    const int64_t L = blockIdx.x, per = nwg / 8;
    const int64_t v = L < 8 * per ? (L % 8) * per + L / 8 : L;
    const int64_t ct = v % gc, rtile = (v / gc) % gr, split = v / (gc * gr);
    const int64_t rt0 = rtile * TA, jt0 = ct * TB;
    const int64_t k_begin = 1 + split * lps;
    const int64_t k_end = (k_begin + lps < kmax + 1) ? k_begin + lps : kmax + 1;
    const int64_t nks = (ne + 63) >> 6;
    const int64_t total = (k_end > k_begin ? k_end - k_begin : 0) * nks;
    double *out = partial + split * ne * nrhs;
    if (total == 0) {  // a split past the last lag contributes zeros
        for (int rt = 0; rt < RT; ++rt)
            for (int r = 0; r < 4; ++r)
                for (int j = 0; j < JT; ++j) {
                    const int64_t row = (rt0 + RT * wr + rt) * 16 + 4 * (lane >> 4) + r;
                    const int64_t n = (jt0 + JT * wn + j) * 16 + (lane & 15);
                    if (row < ne && n < nrhs) out[row * nrhs + n] = 0.0;
                }
        return;
    }
    i4_t acc[5][RT][JT];
#pragma unroll
    for (int w = 0; w < 5; ++w)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int j = 0; j < JT; ++j) acc[w][rt][j] = i4_t{0, 0, 0, 0};
    // staging registers: PF sets, step s held in set s % PF; piece p = tid + NT q
    // is 16 bytes (p % 256) of tile p / 256.  Every load is issued
    // unconditionally (tiles past the edge and steps past the end read a valid
    // address and are masked or never stored), so the compiler can count the
    // loads in flight instead of waiting for all of them.
    i4_t sa[PF][QA], sb[PF][QB];
    int64_t lk = k_begin, lkc = 0;  // load cursor
    auto load = [&](int set) {
        const bool in = lk < k_end;
        const int64_t k = in ? lk : k_end - 1, kc = in ? lkc : nks - 1;
        const int8_t *Ab = slabs + (k - 1) * blk;
        const int8_t *Bb = ring + ((head + k - 1) % n_slots) * slot_bytes;
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int p = tid + NT * q, off = (p & 255) * 16;
            const int64_t rt = rt0 + (p >> 8);
            const i4_t v = *reinterpret_cast<const i4_t *>(Ab + ((rt < nrt ? rt : nrt - 1) * nkc + kc) * 4096 + off);
            sa[set][q] = v & (rt < nrt ? -1 : 0);
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int p = tid + NT * q, off = (p & 255) * 16;
            const int64_t jt = jt0 + (p >> 8);
            const i4_t v = *reinterpret_cast<const i4_t *>(Bb + ((jt < nnt ? jt : nnt - 1) * nkc + kc) * 4096 + off);
            sb[set][q] = v & (jt < nnt ? -1 : 0);
        }
        if (++lkc == nks) {
            lkc = 0;
            ++lk;
        }
    };
    auto store = [&](int set, int buf) {
#pragma unroll
        for (int q = 0; q < QA; ++q) As[buf][tid + NT * q] = sa[set][q];
#pragma unroll
        for (int q = 0; q < QB; ++q) Bs[buf][tid + NT * q] = sb[set][q];
    };
    auto flush = [&](int64_t k, bool first) {
        const double *srow = reinterpret_cast<const double *>(slabs + (k - 1) * blk + R * ld * 4);
        const double *scol =
            reinterpret_cast<const double *>(ring + ((head + k - 1) % n_slots) * slot_bytes + P * ld * 4);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = (rt0 + RT * wr + rt) * 16 + 4 * (lane >> 4) + r;
                const double sr = row < ne ? srow[row] : 0.0;
#pragma unroll
                for (int j = 0; j < JT; ++j) {
                    const int64_t n = (jt0 + JT * wn + j) * 16 + (lane & 15);
                    if (row < ne && n < nrhs) {
                        double g = (double)acc[4][rt][j][r];
                        g = g * 0x1p-7 + (double)acc[3][rt][j][r];
                        g = g * 0x1p-7 + (double)acc[2][rt][j][r];
                        g = g * 0x1p-7 + (double)acc[1][rt][j][r];
                        g = g * 0x1p-7 + (double)acc[0][rt][j][r];
                        const double val = sr * scol[n] * g;
                        double *o = out + row * nrhs + n;
                        *o = first ? val : *o + val;
                    }
#pragma unroll
                    for (int w = 0; w < 5; ++w) acc[w][rt][j][r] = 0;
                }
            }
    };
    // steps 0 .. PF - 1 in flight, step 0 in LDS buffer 0
#pragma unroll
    for (int q = 0; q < PF; ++q) load(q);
    store(0, 0);
    __syncthreads();
    int64_t kcur = k_begin, kccur = 0;
    // two steps per iteration so that buffer and register-set indices are static
    for (int64_t t0 = 0; t0 < total; t0 += 2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t t = t0 + u;
            if (t >= total) break;
            load((u + PF) % PF);  // step t + PF; the set of step t was stored one step ago
            i4_t a[RT][4];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int d = 0; d < 4; ++d) a[rt][d] = As[u][(RT * wr + rt) * 256 + d * 64 + lane];
#pragma unroll
            for (int j = 0; j < JT; ++j) {
                i4_t b[4];
#pragma unroll
                for (int d = 0; d < 4; ++d) b[d] = Bs[u][(JT * wn + j) * 256 + d * 64 + lane];
                // digit pairs (a, b) with a + b <= 4, ordered to space the products into one accumulator
#define QHP_I8_PAIR(A_, B_)                                                                   \
    _Pragma("unroll") for (int rt = 0; rt < RT; ++rt) acc[A_ + B_][rt][j] =                  \
        __builtin_amdgcn_mfma_i32_16x16x64_i8(a[rt][A_], b[B_], acc[A_ + B_][rt][j], 0, 0, 0);
                QHP_I8_PAIR(0, 0)
                QHP_I8_PAIR(0, 1)
                QHP_I8_PAIR(0, 2)
                QHP_I8_PAIR(0, 3)
                QHP_I8_PAIR(1, 3)
                QHP_I8_PAIR(1, 0)
                QHP_I8_PAIR(1, 1)
                QHP_I8_PAIR(1, 2)
                QHP_I8_PAIR(2, 2)
                QHP_I8_PAIR(2, 0)
                QHP_I8_PAIR(2, 1)
                QHP_I8_PAIR(3, 1)
                QHP_I8_PAIR(3, 0)
#undef QHP_I8_PAIR
            }
            // keep the LDS store of step t + 1 behind this step's products: hoisted
            // above them it would wait for its loads with nothing left to overlap
            __builtin_amdgcn_sched_barrier(0);
            if (t + 1 < total) store((u + 1) % PF, u ^ 1);
            if (++kccur == nks) {
                flush(kcur, kcur == k_begin);
                kccur = 0;
                ++kcur;
            }
            __syncthreads();
        }
    }
}

// The same products with the operand pieces copied from memory straight into
// LDS (global_load_lds_dwordx4: each wave instruction moves one 1 KB piece,
// lane l's 16 bytes to byte 16 l of the piece), NB LDS buffers and NB - 1
// steps in flight, so no staging registers and no LDS store instructions.
// Tiles past the edge read a clamped valid tile (their products land in rows
// or right-hand sides that are never written out) and steps past the end
// re-read the last step into a buffer that is never used.
template <int RT, int JT, int WR, int WN, int NB>
__global__ __launch_bounds__(64 * WR * WN, 1) void k_hist_i8d(int64_t ne, int64_t ld, int64_t nrhs, int64_t kmax,
                                                              int64_t lps, int64_t nsplit,
                                                              const int8_t *__restrict__ slabs,
                                                              const int8_t *__restrict__ ring, int64_t n_slots,
                                                              int64_t head, double *__restrict__ partial)
{
    constexpr int NW = WR * WN;                  // waves
    constexpr int TA = RT * WR, TB = JT * WN;    // tiles per step
    constexpr int PIECES = 4 * (TA + TB);        // 1 KB pieces per step
    constexpr int PW = PIECES / NW;              // pieces per wave and step
    static_assert(PW * NW == PIECES, "pieces must divide over the waves");
    constexpr int PF = NB - 1;                   // steps in flight
    __shared__ i4_t S[NB][PIECES * 64];          // [buf][A tiles | B tiles][digit][lane]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave % WR, wn = wave / WR;
    const int64_t R = i8_rows(ne), P = i8_rows(nrhs);
    const int64_t nrt = R >> 4, nnt = P >> 4, nkc = ld >> 6;
    const int64_t blk = i8_block_bytes(ne, ld), slot_bytes = i8_slot_bytes(nrhs, ld);
    const int64_t gr = (nrt + TA - 1) / TA, gc = (nnt + TB - 1) / TB, nwg = gr * gc * nsplit;
    const int64_t L = blockIdx.x, per = nwg / 8;
    const int64_t v = L < 8 * per ? (L % 8) * per + L / 8 : L;
    const int64_t ct = v % gc, rtile = (v / gc) % gr, split = v / (gc * gr);
    const int64_t rt0 = rtile * TA, jt0 = ct * TB;
    const int64_t k_begin = 1 + split * lps;
    const int64_t k_end = (k_begin + lps < kmax + 1) ? k_begin + lps : kmax + 1;
    const int64_t nks = (ne + 63) >> 6;
    const int64_t total = (k_end > k_begin ? k_end - k_begin : 0) * nks;
    double *out = partial + split * ne * nrhs;
    if (total == 0) {
        for (int rt = 0; rt < RT; ++rt)
            for (int r = 0; r < 4; ++r)
                for (int j = 0; j < JT; ++j) {
                    const int64_t row = (rt0 + RT * wr + rt) * 16 + 4 * (lane >> 4) + r;
                    const int64_t n = (jt0 + JT * wn + j) * 16 + (lane & 15);
                    if (row < ne && n < nrhs) out[row * nrhs + n] = 0.0;
                }
        return;
    }
    i4_t acc[5][RT][JT];
#pragma unroll
    for (int w = 0; w < 5; ++w)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int j = 0; j < JT; ++j) acc[w][rt][j] = i4_t{0, 0, 0, 0};
    int64_t lk = k_begin, lkc = 0;  // load cursor
    auto load = [&](int buf) {
        const bool in = lk < k_end;
        const int64_t k = in ? lk : k_end - 1, kc = in ? lkc : nks - 1;
        const int8_t *Ab = slabs + (k - 1) * blk;
        const int8_t *Bb = ring + ((head + k - 1) % n_slots) * slot_bytes;
#pragma unroll
        for (int q = 0; q < PW; ++q) {
            const int pc = wave + NW * q, tile = pc >> 2, d = pc & 3;
            const int8_t *src;
            if (tile < TA) {
                const int64_t rt = rt0 + tile;
                src = Ab + (((rt < nrt ? rt : nrt - 1) * nkc + kc) * 4 + d) * 1024;
            } else {
                const int64_t jt = jt0 + tile - TA;
                src = Bb + (((jt < nnt ? jt : nnt - 1) * nkc + kc) * 4 + d) * 1024;
            }
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const void *>(src + lane * 16),
                                             (__attribute__((address_space(3))) void *)(&S[buf][pc * 64]), 16, 0, 0);
        }
        if (++lkc == nks) {
            lkc = 0;
            ++lk;
        }
    };
    auto flush = [&](int64_t k, bool first) {
        const double *srow = reinterpret_cast<const double *>(slabs + (k - 1) * blk + R * ld * 4);
        const double *scol =
            reinterpret_cast<const double *>(ring + ((head + k - 1) % n_slots) * slot_bytes + P * ld * 4);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = (rt0 + RT * wr + rt) * 16 + 4 * (lane >> 4) + r;
                const double sr = row < ne ? srow[row] : 0.0;
#pragma unroll
                for (int j = 0; j < JT; ++j) {
                    const int64_t n = (jt0 + JT * wn + j) * 16 + (lane & 15);
                    if (row < ne && n < nrhs) {
                        double g = (double)acc[4][rt][j][r];
                        g = g * 0x1p-7 + (double)acc[3][rt][j][r];
                        g = g * 0x1p-7 + (double)acc[2][rt][j][r];
                        g = g * 0x1p-7 + (double)acc[1][rt][j][r];
                        g = g * 0x1p-7 + (double)acc[0][rt][j][r];
                        const double val = sr * scol[n] * g;
                        double *o = out + row * nrhs + n;
                        *o = first ? val : *o + val;
                    }
#pragma unroll
                    for (int w = 0; w < 5; ++w) acc[w][rt][j][r] = 0;
                }
            }
    };
    // vmcnt(n) with the other counters left alone (gfx9 encoding)
    constexpr int WAIT_INFLIGHT = ((PW * (PF - 1)) & 15) | (7 << 4) | (15 << 8) | (((PW * (PF - 1)) >> 4) << 14);
#pragma unroll
    for (int q = 0; q < PF; ++q) load(q);
    __builtin_amdgcn_s_waitcnt(WAIT_INFLIGHT);  // step 0 is in
    __syncthreads();
    int64_t kcur = k_begin, kccur = 0;
    for (int64_t t0 = 0; t0 < total; t0 += NB) {
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int64_t t = t0 + u;
            if (t >= total) break;
            const int buf = u;  // t0 is a multiple of NB
            // step t + PF into the buffer read one step ago (every wave is past it)
            load((u + PF) % NB);
            i4_t a[RT][4];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int d = 0; d < 4; ++d) a[rt][d] = S[buf][((RT * wr + rt) * 4 + d) * 64 + lane];
#pragma unroll
            for (int j = 0; j < JT; ++j) {
                i4_t b[4];
#pragma unroll
                for (int d = 0; d < 4; ++d) b[d] = S[buf][((TA + JT * wn + j) * 4 + d) * 64 + lane];
#define QHP_I8_PAIR(A_, B_)                                                                   \
    _Pragma("unroll") for (int rt = 0; rt < RT; ++rt) acc[A_ + B_][rt][j] =                  \
        __builtin_amdgcn_mfma_i32_16x16x64_i8(a[rt][A_], b[B_], acc[A_ + B_][rt][j], 0, 0, 0);
                QHP_I8_PAIR(0, 0)
                QHP_I8_PAIR(0, 1)
                QHP_I8_PAIR(0, 2)
                QHP_I8_PAIR(0, 3)
                QHP_I8_PAIR(1, 3)
                QHP_I8_PAIR(1, 0)
                QHP_I8_PAIR(1, 1)
                QHP_I8_PAIR(1, 2)
                QHP_I8_PAIR(2, 2)
                QHP_I8_PAIR(2, 0)
                QHP_I8_PAIR(2, 1)
                QHP_I8_PAIR(3, 1)
                QHP_I8_PAIR(3, 0)
#undef QHP_I8_PAIR
            }
            if (++kccur == nks) {
                flush(kcur, kcur == k_begin);
                kccur = 0;
                ++kcur;
            }
            // this wave's pieces of step t + 1 are in; then every wave's are (a
            // plain barrier: the wait above is the only one these copies need)
            __builtin_amdgcn_s_waitcnt(WAIT_INFLIGHT);
            __builtin_amdgcn_s_barrier();
        }
    }
    // the copies issued past the last step land before the wave ends: vmcnt(0)
    __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));
}

// variants of the int8 history kernel (autotuned): wave tile, work-group
// shape, steps prefetched into registers
struct I8Variant {
    int rt, jt, wr, wn, pf, dma;  // dma: pieces copied straight into pf + 1 LDS buffers
};
static const I8Variant kI8[] = {{2, 2, 4, 2, 2, 0}, {2, 2, 4, 2, 1, 1}, {2, 2, 4, 2, 2, 1}};
constexpr int kNumI8 = sizeof(kI8) / sizeof(kI8[0]);
int i8_variant_count() { return kNumI8; }
void i8_variant_desc(int v, int *rows, int *cols, int *waves, int *pf, int *dma)
{
    *rows = 16 * kI8[v].rt * kI8[v].wr;
    *cols = 16 * kI8[v].jt * kI8[v].wn;
    *waves = kI8[v].wr * kI8[v].wn;
    *pf = kI8[v].pf;
    *dma = kI8[v].dma;
}
static const int kI8Default = 2;

int i8_hist_splits(int64_t ne, int64_t kmax, int64_t nrhs, int variant)
{
    // one resident work-group per CU (256 CUs): pick the lags per split that
    // minimise rounds x lags, preferring fewer splits on ties
    if (variant < 0 || variant >= kNumI8) variant = kI8Default;
    const I8Variant &c = kI8[variant];
    const int64_t tiles = ((i8_rows(ne) / 16 + c.rt * c.wr - 1) / (c.rt * c.wr)) *
                          ((i8_rows(nrhs) / 16 + c.jt * c.wn - 1) / (c.jt * c.wn));
    if (kmax < 1) return 1;
    int64_t best_l = 1, best_cost = -1;
    for (int64_t l = 1; l <= kmax; ++l) {
        const int64_t ns = (kmax + l - 1) / l;
        const int64_t cost = ((tiles * ns + 255) / 256) * l;
        if (best_cost < 0 || cost <= best_cost) {
            best_cost = cost;
            best_l = l;
        }
    }
    return (int)((kmax + best_l - 1) / best_l);
}

void launch_hist_i8(hipStream_t s, int64_t ne, int64_t ld, int64_t nrhs, int64_t kmax, int nsplit,
                    const int8_t *slabs, const int8_t *ring, int64_t n_slots, int64_t head, double *partial,
                    int variant)
{
    if (variant < 0 || variant >= kNumI8) variant = kI8Default;
    const I8Variant &c = kI8[variant];
    const int64_t lps = (kmax + nsplit - 1) / nsplit;
    const int64_t nwg = (int64_t)nblk8(i8_rows(ne) / 16, c.rt * c.wr) * nblk8(i8_rows(nrhs) / 16, c.jt * c.wn) * nsplit;
#define QHP_I8_CASE(IDX, KERNEL, A, B, C, D, E)                                                              \
    case IDX:                                                                                                 \
        hipLaunchKernelGGL((KERNEL<A, B, C, D, E>), dim3((unsigned)nwg), dim3(64 * C * D), 0, s, ne, ld, nrhs,    \
                           kmax, lps, (int64_t)nsplit, slabs, ring, n_slots, head, partial);                  \
        break;
    switch (variant) {
        QHP_I8_CASE(0, k_hist_i8, 2, 2, 4, 2, 2)
        QHP_I8_CASE(1, k_hist_i8d, 2, 2, 4, 2, 2)
        default:
        QHP_I8_CASE(2, k_hist_i8d, 2, 2, 4, 2, 3)
    }
#undef QHP_I8_CASE
}

}  // namespace qhp
