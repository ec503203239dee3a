// Lag-banded storage of the raw lag matrices and the factored history
// product (see factored.h).
#include "factored.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

namespace qhp {

static unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

namespace {

constexpr int CW = kBandChunk;  // columns of a chunk
constexpr int META = 4 * 64;    // bytes of a group's words

// value (k, r, c) of a family in stored order: rows r < split from a, the
// others from b (row r - split), through the row and column orders rp, cp
struct Src {
    const double *a, *b;
    const int32_t *rp, *cp;
    int64_t split, lag_stride, row_stride, lag0;
    __device__ double at(int64_t k, int64_t r, int64_t c) const
    {
        const double *p = r < split ? a + (int64_t)rp[r] * row_stride : b + (int64_t)rp[r - split] * row_stride;
        return p[(k - lag0) * lag_stride + cp[c]];
    }
};

// stored value of a pair at one lag: FP64 as is, or FP32 of value + carry
// with the rounding carried to the next lag
__device__ __forceinline__ double store_value(double v, double &carry, bool fp32)
{
    if (!fp32) return v;
    const double t = v + carry;
    const float st = (float)t;
    carry = t - (double)st;
    return (double)st;
}

// lane l of group (q, ch): row 2q + l / CW, column CW ch + l % CW
__device__ __forceinline__ bool group_pair(int64_t g, int64_t nch, int64_t rows, int64_t cols, int lane, int64_t &r,
                                           int64_t &col)
{
    r = 2 * (g / nch) + lane / CW;
    col = (g % nch) * CW + lane % CW;
    return r < rows && col < cols;
}

}  // namespace

// one wave per group: per pair (lane) the first stored lag and the number of
// lags to the last stored value (word klo | len << 16; lags kfirst..lag1, the
// carried rounding from lag0 on); per group the values stored, the lag range
// and the longest run
__global__ __launch_bounds__(256) void k_band_scan(int64_t rows, int64_t cols, int64_t nch, int64_t ng, int64_t lag1,
                                                   int64_t kfirst, Src src, bool fp32, uint32_t *meta,
                                                   int64_t *cnt_out, int32_t *kmin_out, int32_t *kmax_out,
                                                   int32_t *lmax_out)
{
    const int lane = threadIdx.x & 63;
    const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    if (g >= ng) return;
    int64_t r, col;
    const bool in = group_pair(g, nch, rows, cols, lane, r, col);
    double carry = 0.0;
    int64_t first = -1, last = -1;
    if (in)
        for (int64_t k = src.lag0; k <= lag1; ++k)
            if (store_value(src.at(k, r, col), carry, fp32) != 0.0 && k >= kfirst) {
                if (first < 0) first = k;
                last = k;
            }
    const int64_t len = first < 0 ? 0 : last - first + 1;
    meta[g * 64 + lane] = (uint32_t)(first < 0 ? 0 : first) | ((uint32_t)len << 16);
    int64_t c = len, lo = first < 0 ? (1 << 30) : first, hi = last, lm = len;
    for (int off = 32; off > 0; off >>= 1) {
        c += __shfl_xor(c, off, 64);
        lo = min(lo, __shfl_xor(lo, off, 64));
        hi = max(hi, __shfl_xor(hi, off, 64));
        lm = max(lm, __shfl_xor(lm, off, 64));
    }
    if (lane == 0) {
        cnt_out[g] = c;
        kmin_out[g] = (int32_t)(hi < 0 ? 0 : lo);
        kmax_out[g] = (int32_t)hi;
        lmax_out[g] = (int32_t)lm;
    }
}

// one wave per group: the 64 words, then each pair's values over its lags, at
// the group's offset in stored order (row block of qpb groups, chunk, group)
__global__ __launch_bounds__(256) void k_band_fill(int64_t rows, int64_t cols, int64_t nch, int64_t ng, int64_t qpb,
                                                   Src src, bool fp32, const uint64_t *hdr, const uint32_t *meta,
                                                   char *stream)
{
    const int lane = threadIdx.x & 63;
    const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    if (g >= ng) return;
    const int64_t q = g / nch, ch = g % nch;
    const uint64_t h = hdr[((q / qpb) * nch + ch) * qpb + q % qpb];
    if ((h >> 40) == 0) return;  // no stored value in the group
    int64_t r, col;
    group_pair(g, nch, rows, cols, lane, r, col);
    char *base = stream + (h & ((1ull << 40) - 1)) * 16;
    const uint32_t w = meta[g * 64 + lane];
    const int64_t klo = w & 0xffff, len = w >> 16;
    reinterpret_cast<uint32_t *>(base)[lane] = w;
    int64_t start = len;  // exclusive prefix sum of the lengths over the lanes
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t t = __shfl_up(start, off, 64);
        if (lane >= off) start += t;
    }
    start -= len;
    double *v64 = reinterpret_cast<double *>(base + META) + start;
    float *v32 = reinterpret_cast<float *>(base + META) + start;
    double carry = 0.0;
    for (int64_t k = src.lag0; k < klo + len; ++k) {
        const double st = store_value(src.at(k, r, col), carry, fp32);
        if (k < klo) continue;
        if (fp32) v32[k - klo] = (float)st;
        else v64[k - klo] = st;
    }
}

// the work-group shapes the product kernel is built for: waves, and 1 KB
// copy pieces per batch (two batch buffers a wave, 160 KB of LDS at most);
// the 2-wave shapes take the groups of very long runs (coarse meshes)
static const int kBandWaves[] = {16, 12, 8, 4, 2};
static const int kBandPieces[] = {2, 3, 4, 5, 6, 8, 10, 12, 14, 16, 20, 24, 32};
static bool band_shape_built(int w, int p)
{
    bool listed = false;
    for (int q : kBandPieces) listed = listed || q == p;
    for (int v : kBandWaves)
        if (v == w) return listed && 2 * w * p <= 160;
    return false;
}

// rows of the staged x: the tile lags (and for a pass of `block` steps the
// block - 1 lags before them), then zero rows that a lane stepping past its
// run may read.  A lane reads rows klo - tk0 + p + j for p below the longest
// run mx rounded up to a step and j < kBandStep + block - 1; with
// klo - tk0 <= ntk - len (len >= 1) or klo = tk0 (len = 0) the last row read
// is below tmax + lmax + kBandStep + block - 3
static int band_xrows(int tmax, int lmax, int block) { return tmax + lmax + kBandStep + block - 3; }

// LDS bytes of the product kernel: the staged x, two batch buffers a wave,
// the values a lane may read past the last buffer
static size_t band_lds(int tmax, int lmax, int waves, int np, bool fp32, int block)
{
    return (size_t)band_xrows(tmax, lmax, block) * CW * sizeof(double) + (size_t)waves * 2 * np * 1024 +
           (size_t)(lmax + kBandStep) * (fp32 ? 4 : 8);
}

// chunk splits of the product: one work-group per CU (the LDS holds one), at
// least four rounds of them over the 256 CUs, the last round as full as it
// can be (fraction of busy work-group slots), then the fewest work-groups
static int band_splits(int64_t nrb, int64_t nch)
{
    constexpr int64_t kCUs = 256;
    if (nrb * nch <= 4 * kCUs) return (int)nch;
    int best = 1;
    double best_eff = -1.0;
    int64_t best_n = 0;
    for (int64_t ns = 1; ns <= nch; ++ns) {
        const int64_t cps = (nch + ns - 1) / ns, real = (nch + cps - 1) / cps;  // splits that hold chunks
        const int64_t n = nrb * real;
        if (n < 4 * kCUs || real != ns) continue;
        if (n > 8 * kCUs) break;
        const double eff = (double)n / (double)(((n + kCUs - 1) / kCUs) * kCUs);
        if (eff > best_eff + 1e-9 || (eff > best_eff - 1e-9 && n < best_n)) {
            best = (int)ns;
            best_eff = eff;
            best_n = n;
        }
    }
    if (best_eff < 0) return (int)std::max<int64_t>(1, std::min<int64_t>(nch, (4 * kCUs + nrb - 1) / nrb));
    return best;
}

// The group stream of a band read back and rewritten as row lists: row r =
// 2q + h takes, chunk by chunk, the runs of lanes 32h .. 32h + 31 of group
// (q, chunk), lag by lag; the values are copied unchanged.
static void to_row_lists(hipStream_t s, Band &b, bool fp32, const std::vector<uint64_t> &hdr, int64_t qpb)
{
    const int64_t nq = (b.rows + 1) / 2, nch = b.nch;
    const size_t vsz = fp32 ? 4 : 8;
    std::vector<char> st(b.bytes);
    if (b.bytes)
        hip_check(hipMemcpyAsync(st.data(), b.stream.p, b.bytes, hipMemcpyDeviceToHost, s), "band stream");
    hip_check(hipStreamSynchronize(s), "band stream");
    std::vector<int64_t> rptr(b.rows + 1, 0);
    std::vector<char> val;
    std::vector<uint32_t> code;
    val.reserve((size_t)b.nnz * vsz);
    code.reserve((size_t)b.nnz);
    for (int64_t q = 0; q < nq; ++q)
        for (int hf = 0; hf < 2; ++hf) {
            const int64_t r = 2 * q + hf;
            if (r >= b.rows) break;
            for (int64_t ch = 0; ch < nch; ++ch) {
                const uint64_t h = hdr[((q / qpb) * nch + ch) * qpb + q % qpb];
                if ((h >> 40) == 0) continue;
                const char *g = st.data() + (h & ((1ull << 40) - 1)) * 16;
                const uint32_t *w = reinterpret_cast<const uint32_t *>(g);
                int64_t start = 0;
                for (int l = 0; l < 64; ++l) {
                    const int64_t klo = w[l] & 0xffff, len = w[l] >> 16;
                    if (l / CW == hf)
                        for (int64_t p = 0; p < len; ++p) {
                            const char *v = g + META + (start + p) * vsz;
                            val.insert(val.end(), v, v + vsz);
                            code.push_back((uint32_t)((ch * CW + l % CW) << 4 | (klo + p)));
                        }
                    start += len;
                }
            }
            rptr[r + 1] = (int64_t)code.size();
        }
    if ((int64_t)code.size() != b.nnz) throw Fail{QHP_EINVAL, "near band: row lists do not hold every value"};
    b.stream.release();
    b.hdr.release();
    b.clist.release();
    b.clen.release();
    upload(b.rptr, rptr, s);
    b.rval.alloc(std::max<size_t>(val.size(), 16));
    if (!val.empty())
        hip_check(hipMemcpyAsync(b.rval.p, val.data(), val.size(), hipMemcpyHostToDevice, s), "row lists");
    upload(b.rcode, code, s);
    hip_check(hipStreamSynchronize(s), "row lists");
    b.bytes = val.size() + code.size() * 4 + rptr.size() * 8;
}

void build_band(hipStream_t s, int64_t rows, int64_t cols, int64_t lag0, int64_t lag1, const double *srcA,
                const double *srcB, int64_t split, int64_t lag_stride, int64_t row_stride, const int32_t *rp,
                const int32_t *cp, bool fp32, Band &out, int64_t kfirst, int block)
{
    if (lag1 >= 65535) throw Fail{QHP_EINVAL, "the factored history takes at most 65534 lags"};
    if (block != 1 && block != kBandBlock) throw Fail{QHP_EINVAL, "band pass of an unsupported step count"};
    if (kfirst < 0) kfirst = lag0;
    if (block > 1 && kfirst < block) throw Fail{QHP_EINVAL, "a pass of several steps takes lags >= its steps"};
    out.rows = rows;
    out.cols = cols;
    out.nch = (cols + CW - 1) / CW;
    out.lag0 = kfirst;
    out.lag1 = lag1;
    out.block = block;
    const int64_t nq = (rows + 1) / 2, nch = out.nch, ng = nq * nch;
    const size_t vsz = fp32 ? 4 : 8;
    Src src{srcA, srcB, rp, cp, split, lag_stride, row_stride, lag0};
    DBuf meta, cnt, kmin, kmax, lmax;
    meta.alloc(sizeof(uint32_t) * 64 * ng);
    cnt.alloc(sizeof(int64_t) * ng);
    kmin.alloc(sizeof(int32_t) * ng);
    kmax.alloc(sizeof(int32_t) * ng);
    lmax.alloc(sizeof(int32_t) * ng);
    hipLaunchKernelGGL(k_band_scan, dim3(nblk(ng * 64, 256)), dim3(256), 0, s, rows, cols, nch, ng, lag1, kfirst, src,
                       fp32, meta.as<uint32_t>(), cnt.as<int64_t>(), kmin.as<int32_t>(), kmax.as<int32_t>(),
                       lmax.as<int32_t>());
    std::vector<int64_t> hc(ng);
    std::vector<int32_t> hlo(ng), hhi(ng), hlm(ng);
    hip_check(hipMemcpyAsync(hc.data(), cnt.p, sizeof(int64_t) * ng, hipMemcpyDeviceToHost, s), "band scan");
    hip_check(hipMemcpyAsync(hlo.data(), kmin.p, sizeof(int32_t) * ng, hipMemcpyDeviceToHost, s), "band scan");
    hip_check(hipMemcpyAsync(hhi.data(), kmax.p, sizeof(int32_t) * ng, hipMemcpyDeviceToHost, s), "band scan");
    hip_check(hipMemcpyAsync(hlm.data(), lmax.p, sizeof(int32_t) * ng, hipMemcpyDeviceToHost, s), "band scan");
    hip_check(hipStreamSynchronize(s), "band scan");
    std::vector<size_t> gbytes(ng);
    int64_t nnz = 0;
    size_t gmax = 0, gsum = 0;
    int lm = 0;
    for (int64_t g = 0; g < ng; ++g) {
        gbytes[g] = hc[g] ? (META + hc[g] * vsz + 15) / 16 * 16 : 0;
        nnz += hc[g];
        gmax = std::max(gmax, gbytes[g]);
        gsum += gbytes[g];
        lm = std::max(lm, hlm[g]);
    }
    // the lags the groups of a row block of qpb groups use in each chunk
    auto tiles = [&](int64_t qpb, std::vector<uint32_t> &tile) {
        const int64_t nrb = (nq + qpb - 1) / qpb;
        tile.assign(nrb * nch, 0u);
        int tmax = 1;
        for (int64_t rb = 0; rb < nrb; ++rb)
            for (int64_t ch = 0; ch < nch; ++ch) {
                int64_t lo = 1 << 30, hi = -1;
                for (int64_t q = rb * qpb; q < std::min<int64_t>((rb + 1) * qpb, nq); ++q) {
                    const int64_t g = q * nch + ch;
                    if (hhi[g] < 0) continue;
                    lo = std::min<int64_t>(lo, hlo[g]);
                    hi = std::max<int64_t>(hi, hhi[g]);
                }
                if (hi < 0) continue;
                tile[rb * nch + ch] = (uint32_t)lo | ((uint32_t)(hi - lo + 1) << 16);
                tmax = std::max<int>(tmax, (int)(hi - lo + 1));
            }
        return tmax;
    };
    // work-group shape: the most bytes in flight (waves x 1 KB copy pieces
    // per batch), counted in full from 8 waves on and in proportion below
    // (fewer waves hide less latency), then the most waves, whose buffers and
    // staged x fit the LDS; a batch holds at least the largest group
    const int npmin = (int)((gmax + 1023) / 1024);
    // a small band (a few hundred KB a CU) is bound by each work-group's
    // latency, not by bytes in flight: 8 waves and the smallest batch that
    // holds the largest group, so that several work-groups share a CU
    const bool small = gsum < ((size_t)64 << 20);
    std::vector<uint32_t> tile, tw;
    int waves = 0, np = 0, tmax = 0;
    for (int w : kBandWaves) {
        if (small && w != 8 && waves) continue;
        const int tm = tiles((int64_t)w * band_groups_per_wave(block, w), tw);
        int p = 0;  // the largest batch built for this size that fits (small: the smallest that holds a group)
        for (int q : kBandPieces)
            if (band_shape_built(w, q) && band_lds(tm, lm, w, q, fp32, block) <= (size_t)kBandLdsBytes &&
                (!small || !p || p < npmin))
                p = q;
        if (p < npmin) continue;
        if (small) {
            if (!waves || w == 8) {
                waves = w;
                np = p;
                tmax = tm;
                tile = tw;
            }
            continue;
        }
        // a pass of several steps does several products per value: its walk
        // needs more waves to hide, counted in full up to 16 (two groups a wave
        // at 16 waves keep the kBandBlock sums a row within 128 registers)
        auto score = [&](int w_, int p_) { return w_ * p_ * std::min(w_, block > 1 ? 16 : 8); };
        if (!waves || score(w, p) > score(waves, np)) {
            waves = w;
            np = p;
            tmax = tm;
            tile = tw;
        }
    }
    if (std::getenv("QHP_VERBOSE")) {  // distribution of group sizes and tile lag ranges
        std::vector<size_t> gs;
        for (size_t b : gbytes)
            if (b) gs.push_back(b);
        std::sort(gs.begin(), gs.end());
        std::vector<int> tr;
        for (uint32_t t : tile)
            if (t >> 16) tr.push_back((int)(t >> 16));
        std::sort(tr.begin(), tr.end());
        if (!gs.empty() && !tr.empty())
            std::fprintf(stderr,
                         "[qhp]   group bytes p50 %zu p99 %zu max %zu; longest run %d; tile lag range p50 %d p90 %d "
                         "max %d\n",
                         gs[gs.size() / 2], gs[gs.size() * 99 / 100], gs.back(), lm, tr[tr.size() / 2],
                         tr[tr.size() * 9 / 10], tr.back());
    }
    if (!waves) throw Fail{QHP_EINVAL, "factored history: a band group does not fit the LDS"};
    const int64_t qpb = (int64_t)waves * band_groups_per_wave(block, waves);
    out.nrb = (nq + qpb - 1) / qpb;
    // offsets in stored order: row block, chunk, group (the headers of a
    // wave's groups in one chunk are consecutive)
    std::vector<uint64_t> hdr(out.nrb * nch * qpb, 0);
    uint64_t off = 0;
    for (int64_t rb = 0; rb < out.nrb; ++rb)
        for (int64_t ch = 0; ch < nch; ++ch)
            for (int64_t i = 0; i < qpb; ++i) {
                const int64_t q = rb * qpb + i;
                const size_t b = q < nq ? gbytes[q * nch + ch] : 0;
                hdr[(rb * nch + ch) * qpb + i] = (off / 16) | ((uint64_t)(b / 16) << 40);
                off += b;
            }
    if (off / 16 >= (1ull << 40)) throw Fail{QHP_ENOMEM, "factored history stream too large"};
    out.bytes = off;
    out.nnz = nnz;
    out.tmax = tmax;
    out.lmax = lm;
    out.waves = waves;
    out.np = np;
    upload(out.hdr, hdr, s);
    upload(out.tile, tile, s);
    // per row block the chunks whose tile holds lags (the others have no value)
    std::vector<int32_t> clist(out.nrb * nch, 0), clen(out.nrb, 0);
    out.cmax = 0;
    for (int64_t rb = 0; rb < out.nrb; ++rb) {
        for (int64_t ch = 0; ch < nch; ++ch)
            if (tile[rb * nch + ch] >> 16) clist[rb * nch + clen[rb]++] = (int32_t)ch;
        out.cmax = std::max<int64_t>(out.cmax, clen[rb]);
    }
    upload(out.clist, clist, s);
    upload(out.clen, clen, s);
    // a batch's copy reads np whole 1 KB pieces from its first group on
    out.stream.alloc(off + (size_t)np * 1024 + 1024);
    hip_check(hipMemsetAsync(out.stream.p, 0, off + (size_t)np * 1024 + 1024, s), "stream");
    hipLaunchKernelGGL(k_band_fill, dim3(nblk(ng * 64, 256)), dim3(256), 0, s, rows, cols, nch, ng, qpb, src, fp32,
                       out.hdr.as<uint64_t>(), meta.as<uint32_t>(), out.stream.as<char>());
    hip_check(hipStreamSynchronize(s), "band fill");
    out.nsplit = out.cmax ? band_splits(out.nrb, out.cmax) : 1;
    // a one-step band (the near lags): row lists, one partial
    out.direct = block == 1;
    if (out.direct) {
        if (lag1 >= 16 || cols >= (1ll << 28)) throw Fail{QHP_EINVAL, "near band too wide for its row lists"};
        out.nsplit = 1;
        to_row_lists(s, out, fp32, hdr, qpb);
    }
}

namespace {

// inclusive sum and maximum over the wave's 64 lanes (DPP row shifts within
// rows of 16 lanes, then the row broadcasts); all lanes active
template <int CTRL, int RMASK>
__device__ __forceinline__ int dpp_add(int v)
{
    return v + __builtin_amdgcn_update_dpp(0, v, CTRL, RMASK, 0xf, true);
}
__device__ __forceinline__ int wave_incl_sum(int v)
{
    v = dpp_add<0x111, 0xf>(v);  // row_shr:1
    v = dpp_add<0x112, 0xf>(v);  // row_shr:2
    v = dpp_add<0x114, 0xf>(v);  // row_shr:4
    v = dpp_add<0x118, 0xf>(v);  // row_shr:8
    v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
    v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3
    return v;
}
__device__ __forceinline__ int wave_max_nonneg(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true));
    const int a = max(__builtin_amdgcn_readlane(v, 15), __builtin_amdgcn_readlane(v, 31));
    const int b = max(__builtin_amdgcn_readlane(v, 47), __builtin_amdgcn_readlane(v, 63));
    return max(a, b);
}

// a stored value as FP64, or zero when !keep (an FP32 value is cleared as
// bits, before the conversion: one 32-bit select; the empty asm keeps the
// compiler from moving the select past the conversion, where it takes two)
__device__ __forceinline__ double masked(float v, bool keep)
{
    uint32_t b = keep ? __float_as_uint(v) : 0u;
    asm("" : "+v"(b));
    return (double)__uint_as_float(b);
}
__device__ __forceinline__ double masked(double v, bool keep) { return keep ? v : 0.0; }

// work-group barrier for data shared through LDS only: the wave's LDS
// accesses complete (lgkmcnt(0)), then s_barrier; global loads and copies in
// flight stay in flight (a __syncthreads fence waits for them too).  The
// empty asm statements keep the compiler from moving memory accesses across.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt((15) | (7 << 4) | (0 << 8) | (3 << 14));  // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// s_waitcnt vmcnt(N), lgkmcnt and expcnt left alone
template <int N>
__device__ __forceinline__ void wait_vm()
{
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

}  // namespace

// The banded product.  A work-group is W waves; wave w takes the
// kBandRowsPerWave / 2 groups (row pairs) rb * W * 8 + 8 w + [0, 8) of row
// block rb, over one split of the chunks.  Per chunk the work-group stages x_k
// of the chunk's CW columns for the tile's lags into LDS ([lag][column], FP64;
// the rows past them zero).  Each wave streams its groups, chunk after chunk,
// in batches: as many consecutive groups as fit np 1 KB pieces (one
// contiguous range), copied straight into one of its two LDS batch buffers
// (global_load_lds, 16 bytes a lane, always np pieces so the waits are
// exact); while it walks one batch the next is in flight.  In a group lane l
// takes pair l: its words give the run (klo, len), a wave prefix sum its
// place among the values; the wave steps over the longest run kBandStep lags
// at a time, a lane past its own run adding zero products.  FP64 sums per lane,
// reduced over each half-wave (one row) at the end, one partial per split.
// A pass of BB steps stages the BB - 1 lags before the tile too and forms, for
// each value of lag k, its products with the staged lags k - b (b < BB): the
// sums of the steps b after the current one.
template <typename T, int W, int NP, int BB>
__global__ __launch_bounds__(64 * W) void k_band(int64_t rows, int64_t nch, int64_t cps,
                                                 const uint64_t *__restrict__ hdr, const uint32_t *__restrict__ tile,
                                                 const int32_t *__restrict__ clist, const int32_t *__restrict__ clen,
                                                 const char *__restrict__ stream, const double *__restrict__ x,
                                                 int64_t ldx, int64_t K, int64_t head, int64_t slot0, int xrows,
                                                 double *__restrict__ part)
{
    constexpr int GW = band_groups_per_wave(BB, W);  // groups (row pairs) of a wave in a chunk
    extern __shared__ double smem[];
    double *X = smem;
    // the wave index is uniform: group quantities below stay in scalar registers
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col = lane & (CW - 1);
    constexpr int64_t batch = (int64_t)NP * 1024;
    char *bufs = reinterpret_cast<char *>(smem + (int64_t)xrows * CW) + (int64_t)wave * 2 * batch;
    const int64_t rb = blockIdx.x, sp = blockIdx.y;
    // chunk positions below index the row block's list of chunks that hold
    // values (CLk: position -> chunk); the split takes cps of them
    typedef const __attribute__((address_space(4))) int32_t *cint_t;
    const cint_t CL = (cint_t)clist, CN = (cint_t)clen;
    auto CLk = [&](int64_t j) { return (int64_t)CL[rb * nch + j]; };
    const int64_t nlist = CN[rb];
    const int64_t c0 = sp * cps, c1 = (c0 + cps < nlist) ? c0 + cps : nlist;
    const int64_t q0w = rb * W * GW + (int64_t)wave * GW;  // first group (row pair) of this wave
    const int64_t nqt = (rows + 1) / 2;
    const int ngw = nqt - q0w < GW ? (int)(nqt - q0w) : GW;  // groups of this wave (may be <= 0)
    double acc[GW][BB];
#pragma unroll
    for (int q = 0; q < GW; ++q)
#pragma unroll
        for (int b = 0; b < BB; ++b) acc[q][b] = 0.0;
    // headers and tiles read through the constant address space: scalar loads,
    // whose waits (lgkmcnt) leave the copies in flight (vmcnt) alone; a wave's
    // headers of one chunk are consecutive
    typedef const __attribute__((address_space(4))) uint64_t *chdr_t;
    typedef const __attribute__((address_space(4))) uint32_t *ctile_t;
    const chdr_t H = (chdr_t)hdr;
    const ctile_t TL = (ctile_t)tile;
    const int64_t qpb = (int64_t)W * GW;
    auto hidx = [&](int64_t ch, int q) { return (rb * nch + CLk(ch)) * qpb + (int64_t)wave * GW + q; };
    auto gsize = [&](int64_t ch, int q) { return q < ngw ? (int64_t)(H[hidx(ch, q)] >> 40) * 16 : 0; };
    // the batch after groups [.., q0) of chunk ch: skip empty groups, then take
    // consecutive groups while they fit the batch; false when none is left
    auto next_batch = [&](int64_t &ch, int &q0, int &q1) {
        while (ch < c1) {
            while (q0 < ngw && gsize(ch, q0) == 0) ++q0;
            if (q0 < ngw) break;
            ++ch;
            q0 = 0;
        }
        if (ch >= c1) return false;
        int64_t total = 0;
        q1 = q0;
        while (q1 < ngw) {
            const int64_t sz = gsize(ch, q1);
            if (total + sz > batch) break;
            total += sz;
            ++q1;
        }
        return true;
    };
    auto issue = [&](int64_t ch, int q0, char *dst) {
        const char *src = stream + (H[hidx(ch, q0)] & ((1ull << 40) - 1)) * 16;
#pragma unroll
        for (int pc = 0; pc < NP; ++pc)
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const void *>(src + pc * 1024 + lane * 16),
                                             (__attribute__((address_space(3))) void *)(dst + pc * 1024), 16, 0, 0);
    };
    // x of a chunk's tile: element idx = lag row idx / CW (lag tk0 - BB + 1 +
    // row), column idx % CW; the first XR * 64 W elements go through
    // registers, loaded a chunk ahead
    constexpr int XR = (kBandPrefetchLags * CW + 64 * W - 1) / (64 * W);
    // lags 1 .. K: head + k - 1 < 2K, one subtraction wraps the ring
    auto x_at = [&](int64_t ch, int tk0, int idx) {
        const int64_t k = tk0 - (BB - 1) + idx / CW, cc = CLk(ch) * CW + idx % CW;
        int64_t slot = k == 0 ? slot0 : head + k - 1;
        if (k != 0 && slot >= K) slot -= K;
        return cc < ldx ? x[slot * ldx + cc] : 0.0;
    };
    double xpre[XR];
    // staged rows of a tile (none for an empty one: its lags would be <= 0)
    auto nrows = [&](int ntk) { return ntk ? ntk + BB - 1 : 0; };
    auto prefetch = [&](int64_t ch, int tk0, int ntk) {
#pragma unroll
        for (int r = 0; r < XR; ++r) {
            const int idx = threadIdx.x + r * 64 * W;
            xpre[r] = idx < nrows(ntk) * CW ? x_at(ch, tk0, idx) : 0.0;
        }
    };
    // zero rows past any tile: read (and discarded) by lanes past their runs
    for (int idx = threadIdx.x; idx < xrows * CW; idx += 64 * W) X[idx] = 0.0;
    uint32_t tl_next = c0 < c1 ? TL[rb * nch + CLk(c0)] : 0u;
    prefetch(c0, (int)(tl_next & 0xffff), (int)(tl_next >> 16));
    int64_t bch = c0;
    int bq0 = 0, bq1 = 0, cur = 0;
    bool have = ngw > 0 && next_batch(bch, bq0, bq1);
    if (have) issue(bch, bq0, bufs);
    for (int64_t ch = c0; ch < c1; ++ch) {
        const uint32_t tl = tl_next;
        const int tk0 = (int)(tl & 0xffff), ntk = (int)(tl >> 16);
        lds_barrier();  // every wave is done with the previous chunk's x
#pragma unroll
        for (int r = 0; r < XR; ++r) {
            const int idx = threadIdx.x + r * 64 * W;
            if (idx < nrows(ntk) * CW) X[idx] = xpre[r];
        }
        for (int idx = threadIdx.x + XR * 64 * W; idx < nrows(ntk) * CW; idx += 64 * W) X[idx] = x_at(ch, tk0, idx);
        lds_barrier();
        if (ch + 1 < c1) {  // the next chunk's x, in flight during this chunk's walk
            tl_next = TL[rb * nch + CLk(ch + 1)];
            prefetch(ch + 1, (int)(tl_next & 0xffff), (int)(tl_next >> 16));
        }
        while (have && bch == ch) {
            int64_t nch_ = bch;
            int nq0 = bq1, nq1 = 0;
            const bool nhave = next_batch(nch_, nq0, nq1);
            if (nhave) {
                issue(nch_, nq0, bufs + (1 - cur) * batch);
                wait_vm<NP>();
            } else {
                wait_vm<0>();
            }
            const char *buf = bufs + cur * batch;
            int64_t goff = 0;
#pragma unroll
            for (int q = 0; q < GW; ++q) {
                if (q < bq0 || q >= bq1) continue;
                const int64_t sz = gsize(ch, q);
                if (sz == 0) continue;
                const char *g = buf + goff;
                goff += sz;
                const uint32_t w = reinterpret_cast<const uint32_t *>(g)[lane];
                const int len = (int)(w >> 16), klo = len ? (int)(w & 0xffff) : tk0;
                const int start = wave_incl_sum(len) - len;
                const int mx = wave_max_nonneg(len);
                const T *vals = reinterpret_cast<const T *>(g + META) + start;
                // row of the lag klo - b + u for the step b after the current one: u + BB - 1 - b
                const double *xr = X + (klo - tk0) * CW + col;
                double sum[BB];
#pragma unroll
                for (int b = 0; b < BB; ++b) sum[b] = 0.0;
                // kBandStep lags a step, every read issued before the
                // products; a lane past its run reads the values after it (in
                // LDS) and zero or staged x rows, and adds zero products.  The
                // x window (rows p .. p + kBandStep + BB - 2) keeps its last
                // BB - 1 rows for the next step, which reads kBandStep new ones
                double xv[kBandStep + BB - 1];
#pragma unroll
                for (int j = 0; j < BB - 1; ++j) xv[j] = xr[j * CW];
                for (int p = 0; p < mx; p += kBandStep) {
                    T v[kBandStep];
#pragma unroll
                    for (int u = 0; u < kBandStep; ++u) v[u] = vals[p + u];
#pragma unroll
                    for (int j = BB - 1; j < kBandStep + BB - 1; ++j) xv[j] = xr[(p + j) * CW];
#pragma unroll
                    for (int u = 0; u < kBandStep; ++u) {
                        const double mv = masked(v[u], p + u < len);
#pragma unroll
                        for (int b = 0; b < BB; ++b) sum[b] = fma(mv, xv[u + BB - 1 - b], sum[b]);
                    }
#pragma unroll
                    for (int j = 0; j < BB - 1; ++j) xv[j] = xv[j + kBandStep];
                }
#pragma unroll
                for (int b = 0; b < BB; ++b) acc[q][b] += sum[b];
            }
            bch = nch_;
            bq0 = nq0;
            bq1 = nq1;
            have = nhave;
            cur = 1 - cur;
        }
        // at most the batch in flight is outstanding (a no-op after a walk):
        // the next chunk's x, loaded before it, is complete
        wait_vm<NP>();
    }
#pragma unroll
    for (int q = 0; q < GW; ++q)
#pragma unroll
        for (int b = 0; b < BB; ++b) {
            double v = acc[q][b];
            for (int off = CW / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            acc[q][b] = v;
        }
    if (col == 0)
#pragma unroll
        for (int q = 0; q < GW; ++q) {
            const int64_t r = 2 * (q0w + q) + lane / CW;
            if (q < ngw && r < rows)
#pragma unroll
                for (int b = 0; b < BB; ++b) part[(sp * BB + b) * rows + r] = acc[q][b];
        }
}

// The product of a band of short runs (at most kBandStep lags, the near
// lags) from its row lists: one wave per row, the lanes over its entries
// (kRowUnroll entries a lane in flight: the values and words, then the x
// they name, which the few ring slots keep in L2), FP64 sums per lane
// reduced over the wave, one partial per row.
constexpr int kRowUnroll = 4;
template <typename T>
__global__ __launch_bounds__(256) void k_band_rows(int64_t rows, const int64_t *__restrict__ rptr,
                                                   const T *__restrict__ val, const uint32_t *__restrict__ code,
                                                   const double *__restrict__ x, int64_t ldx, int64_t K,
                                                   int64_t head, int64_t slot0, double *__restrict__ part)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = __builtin_amdgcn_readfirstlane((int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    if (r >= rows) return;  // whole waves
    const int64_t beg = rptr[r], end = rptr[r + 1];
    double acc = 0.0;
    for (int64_t t0 = beg; t0 < end; t0 += 64 * kRowUnroll) {
        T v[kRowUnroll];
        uint32_t c[kRowUnroll];
        // no branch between the loads: an entry past the row's end loads the
        // row's last one (t0 < end) and is masked to value 0, word 0 (lag 0,
        // column 0: an x inside the ring)
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            const int64_t t = t0 + 64 * u + lane, tc = t < end ? t : end - 1;
            const T vv = val[tc];
            const uint32_t cc = code[tc];
            v[u] = t < end ? vv : T(0);
            c[u] = t < end ? cc : 0u;
        }
        double xv[kRowUnroll];
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            const int64_t k = c[u] & 15, col = c[u] >> 4;
            int64_t slot = k == 0 ? slot0 : head + k - 1;
            if (k != 0 && slot >= K) slot -= K;
            xv[u] = x[slot * ldx + col];
        }
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) acc = fma((double)v[u], xv[u], acc);
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) part[r] = acc;
}

template <typename T, int W, int NP, int BB>
static void band_launch(hipStream_t s, const Band &b, bool fp32, const double *x, int64_t ldx, int64_t K,
                        int64_t head, int64_t slot0, double *part)
{
    const int64_t cps = (b.cmax + b.nsplit - 1) / b.nsplit;
    const size_t lds = band_lds(b.tmax, b.lmax, W, NP, fp32, BB);
    static bool attr = false;
    if (!attr) {
        hip_check(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_band<T, W, NP, BB>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, kBandLdsBytes),
                  "band kernel attribute");
        attr = true;
    }
    const int xrows = band_xrows(b.tmax, b.lmax, BB);
    hipLaunchKernelGGL((k_band<T, W, NP, BB>), dim3((unsigned)b.nrb, (unsigned)b.nsplit), dim3(64 * W), lds, s,
                       b.rows, b.nch, cps, b.hdr.as<uint64_t>(), b.tile.as<uint32_t>(), b.clist.as<int32_t>(),
                       b.clen.as<int32_t>(), b.stream.as<char>(), x, ldx, K, head, slot0, xrows, part);
}

template <typename T, int W, int BB>
static void band_pieces(hipStream_t s, const Band &b, bool fp32, const double *x, int64_t ldx, int64_t K,
                        int64_t head, int64_t slot0, double *part)
{
#define QHP_NP(P)                                                                    \
    if constexpr (2 * W * P <= 160)                                                  \
        if (b.np == P) return band_launch<T, W, P, BB>(s, b, fp32, x, ldx, K, head, slot0, part);
    QHP_NP(2) QHP_NP(3) QHP_NP(4) QHP_NP(5) QHP_NP(6) QHP_NP(8) QHP_NP(10) QHP_NP(12) QHP_NP(14) QHP_NP(16)
    QHP_NP(20) QHP_NP(24) QHP_NP(32)
#undef QHP_NP
    throw Fail{QHP_EINVAL, "band kernel shape not built"};
}

template <typename T, int BB>
static void band_dispatch(hipStream_t s, const Band &b, bool fp32, const double *x, int64_t ldx, int64_t K,
                          int64_t head, int64_t slot0, double *part)
{
    switch (b.waves) {
    case 16:
        return band_pieces<T, 16, BB>(s, b, fp32, x, ldx, K, head, slot0, part);
        break;
    case 12: return band_pieces<T, 12, BB>(s, b, fp32, x, ldx, K, head, slot0, part);
    case 8: return band_pieces<T, 8, BB>(s, b, fp32, x, ldx, K, head, slot0, part);
    case 4: return band_pieces<T, 4, BB>(s, b, fp32, x, ldx, K, head, slot0, part);
    case 2: return band_pieces<T, 2, BB>(s, b, fp32, x, ldx, K, head, slot0, part);
    default: break;
    }
    throw Fail{QHP_EINVAL, "band kernel shape not built"};
}

void launch_band(hipStream_t s, const Band &b, bool fp32, const double *x, int64_t ldx, int64_t K, int64_t head,
                 int64_t slot0, double *part)
{
    if (b.direct) {
        const dim3 grid(nblk(b.rows * 64, 256));
        if (fp32)
            hipLaunchKernelGGL(k_band_rows<float>, grid, dim3(256), 0, s, b.rows, b.rptr.as<int64_t>(),
                               b.rval.as<float>(), b.rcode.as<uint32_t>(), x, ldx, K, head, slot0, part);
        else
            hipLaunchKernelGGL(k_band_rows<double>, grid, dim3(256), 0, s, b.rows, b.rptr.as<int64_t>(),
                               b.rval.as<double>(), b.rcode.as<uint32_t>(), x, ldx, K, head, slot0, part);
        return;
    }
    if (!band_shape_built(b.waves, b.np)) throw Fail{QHP_EINVAL, "band kernel shape not built"};
    if (b.block == kBandBlock) {
        if (fp32) band_dispatch<float, kBandBlock>(s, b, fp32, x, ldx, K, head, slot0, part);
        else band_dispatch<double, kBandBlock>(s, b, fp32, x, ldx, K, head, slot0, part);
    } else {
        throw Fail{QHP_EINVAL, "band pass of an unsupported step count"};
    }
}

__global__ void k_fac_combine(int64_t ne, int64_t nc, const int32_t *cells, const double *area, double T0,
                              const int32_t *einv, const int32_t *cinv, const double *pac, int nsac,
                              const double *ps, int nss, const double *pacf, int nsacf, const double *psf, int nssf,
                              int b, int nb, double *em, int64_t ld)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= ne) return;
    const int64_t cp = cells[2 * m], cm = cells[2 * m + 1], ms = einv[m], cps = cinv[cp], cms = cinv[cm];
    double a = 0.0, c = 0.0, sp = 0.0, sm = 0.0;
    for (int q = 0; q < nsac; ++q) {
        a += pac[q * 2 * ne + ms];
        c += pac[q * 2 * ne + ne + ms];
    }
    for (int q = 0; q < nss; ++q) {
        sp += ps[q * nc + cps];
        sm += ps[q * nc + cms];
    }
    if (pacf) {  // the far lags, from the pass's partials of this step
        for (int q = 0; q < nsacf; ++q) {
            a += pacf[((int64_t)q * nb + b) * 2 * ne + ms];
            c += pacf[((int64_t)q * nb + b) * 2 * ne + ne + ms];
        }
        for (int q = 0; q < nssf; ++q) {
            sp += psf[((int64_t)q * nb + b) * nc + cps];
            sm += psf[((int64_t)q * nb + b) * nc + cms];
        }
    }
    em[m] = a - T0 * (sp / area[cp] - sm / area[cm]);
    em[ld + m] = c;
}

void launch_fac_combine(hipStream_t s, int64_t ne, int64_t nc, const int32_t *cells, const double *area, double T0,
                        const int32_t *einv, const int32_t *cinv, const double *pac, int nsac, const double *ps,
                        int nss, const double *pacf, int nsacf, const double *psf, int nssf, int b, int nb,
                        double *em, int64_t ld)
{
    hipLaunchKernelGGL(k_fac_combine, dim3(nblk(ne, 256)), dim3(256), 0, s, ne, nc, cells, area, T0, einv, cinv, pac,
                       nsac, ps, nss, pacf, nsacf, psf, nssf, b, nb, em, ld);
}

// out[b][e] = sum_s part[s][b][e] (e < n, b < nb), splits summed in order
__global__ void k_sum_splits(int64_t n, int nsplit, int nb, const double *part, double *out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nb) return;
    const int64_t b = e / n, i = e % n;
    double a = 0.0;
    for (int q = 0; q < nsplit; ++q) a += part[((int64_t)q * nb + b) * n + i];
    out[b * n + i] = a;
}

void launch_sum_splits(hipStream_t s, int64_t n, int nsplit, int nb, const double *part, double *out)
{
    hipLaunchKernelGGL(k_sum_splits, dim3(nblk(n * nb, 256)), dim3(256), 0, s, n, nsplit, nb, part, out);
}

__global__ void k_fac_post_a(int64_t nc, const int32_t *tri_edge, const int32_t *tri_sign, const double *area,
                             const int32_t *cinv, const double *y, double *sv, double *cslot)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    double a = 0.0;
    for (int i = 0; i < 3; ++i) a += tri_sign[3 * c + i] * y[tri_edge[3 * c + i]];
    sv[c] = a;
    cslot[cinv[c]] = a / area[c];
}

void launch_fac_post_a(hipStream_t s, int64_t nc, const int32_t *tri_edge, const int32_t *tri_sign,
                       const double *area, const int32_t *cinv, const double *y, double *sv, double *cslot)
{
    hipLaunchKernelGGL(k_fac_post_a, dim3(nblk(nc, 256)), dim3(256), 0, s, nc, tri_edge, tri_sign, area, cinv, y, sv,
                       cslot);
}

__global__ void k_fac_post_b(int64_t ne, double dtn, const int32_t *cells, const int32_t *einv, const double *y,
                             const double *zc, const double *zp, double *jslot, double *j_out, double *x0)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= ne) return;
    const int64_t cp = cells[2 * m], cm = cells[2 * m + 1], ms = einv[m];
    const double vc = zc[cp] - zc[cm], vp = zp[cp] - zp[cm];  // (P^Sigma y_i)_m, (P^Sigma y_{i-1})_m
    const double j = y[m] + (1.0 / dtn - 1.0) * vc - vp / dtn;
    jslot[ms] = j;
    if (j_out) j_out[m] = j;
    x0[ms] = -vc / dtn;
}

void launch_fac_post_b(hipStream_t s, int64_t ne, double dtn, const int32_t *cells, const int32_t *einv,
                       const double *y, const double *zc, const double *zp, double *jslot, double *j_out, double *x0)
{
    hipLaunchKernelGGL(k_fac_post_b, dim3(nblk(ne, 256)), dim3(256), 0, s, ne, dtn, cells, einv, y, zc, zp, jslot,
                       j_out, x0);
}

// 21 bits of each coordinate interleaved (x highest)
static uint64_t morton3(double fx, double fy, double fz)
{
    auto spread = [](uint64_t v) {
        v &= 0x1fffff;
        v = (v | v << 32) & 0x1f00000000ffffull;
        v = (v | v << 16) & 0x1f0000ff0000ffull;
        v = (v | v << 8) & 0x100f00f00f00f00full;
        v = (v | v << 4) & 0x10c30c30c30c30c3ull;
        v = (v | v << 2) & 0x1249249249249249ull;
        return v;
    };
    auto q = [](double f) { return (uint64_t)(std::min(std::max(f, 0.0), 1.0 - 1e-12) * 2097152.0); };
    return spread(q(fx)) << 2 | spread(q(fy)) << 1 | spread(q(fz));
}

void morton_order(const Mesh &m, bool cells, std::vector<int32_t> &perm, std::vector<int32_t> &inv)
{
    const int64_t n = cells ? m.nc : m.ne;
    std::vector<double> p(3 * n);
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            if (cells)
                p[3 * i + k] = (m.xyz[3 * m.tri[3 * i] + k] + m.xyz[3 * m.tri[3 * i + 1] + k] +
                                m.xyz[3 * m.tri[3 * i + 2] + k]) / 3.0;
            else
                p[3 * i + k] = 0.5 * (m.xyz[3 * m.edges[2 * i] + k] + m.xyz[3 * m.edges[2 * i + 1] + k]);
        }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], p[3 * i + k]);
            hi[k] = std::max(hi[k], p[3 * i + k]);
        }
    const double span = std::max(std::max(hi[0] - lo[0], hi[1] - lo[1]), std::max(hi[2] - lo[2], 1e-300));
    std::vector<std::pair<uint64_t, int32_t>> key(n);
    for (int64_t i = 0; i < n; ++i)
        key[i] = {morton3((p[3 * i] - lo[0]) / span, (p[3 * i + 1] - lo[1]) / span, (p[3 * i + 2] - lo[2]) / span),
                  (int32_t)i};
    std::sort(key.begin(), key.end());
    perm.resize(n);
    inv.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        perm[i] = key[i].second;
        inv[key[i].second] = (int32_t)i;
    }
}

}  // namespace qhp
