// The factored history sum (Sec. IV-A, IV-C): instead of the dense blocks
// T_k = P_E W^E_k + P_M W^M_k, the raw lag matrices A_k, C_k (edge pairs)
// and Sq_k, the q_0 combination of the shell moments (triangle pairs, B_k =
// -T0 Sigma diag(1/A) Sq_k diag(1/A) Sigma^T), stored lag-banded, applied to
// the histories of the current j and of the cell charges; the dense P_E, P_M
// once per step.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "ctx.h"

namespace qhp {

// A work-group of the banded product: `waves` waves (16, 12, 8, 4 or 2,
// chosen at build time with the size of the copy batches so that the staged x
// and two batch buffers a wave fit the LDS), each taking kBandRowsPerWave
// rows (one row block) over one split of the kBandChunk-column chunks.
constexpr int kBandRowsPerWave = 16;
constexpr int kBandChunk = 32;
constexpr int kBandLdsBytes = 160 * 1024;
constexpr int kBandStep = 8;        // lags a lane takes per step of the walk
constexpr int kBandPrefetchLags = 128;  // lags of a chunk's x loaded ahead through registers
// steps of one pass over the far lags (k >= kBandBlock): their terms for steps
// i .. i + kBandBlock - 1 use only the currents of steps <= i - 1, so one pass
// over the values at step i gives all of them (each value serves kBandBlock
// products); the near lags (k < kBandBlock) are applied every step
constexpr int kBandBlock = 8;
// groups (row pairs) a wave takes in a chunk: fewer in a pass of several
// steps, whose sums per row multiply with the steps, and fewer again from 12
// waves a work-group on (at 16 waves, four waves a SIMD: at most 128
// registers a lane)
constexpr int band_groups_per_wave(int block, int waves)
{
    return block > 4 ? (waves >= 12 ? 2 : 4) : kBandRowsPerWave / 2;
}

// One lag-banded family of matrices X_k, k in [lag0, lag1], rows x cols.
// Rows 2q, 2q + 1 and the chunk ch of kBandChunk columns form the group
// g = q * nch + ch, 64 pairs (lane l: row 2q + l / kBandChunk, column
// kBandChunk ch + l % kBandChunk): for each pair the lags from its first to
// its last stored value.  A group is 64 words klo | len << 16, then the
// values, pair by pair, lag by lag within a pair: FP64, or FP32 with the
// rounding of each pair carried from lag to lag; padded to 16 bytes.  Groups
// are stored by row block (waves * kBandRowsPerWave / 2 groups), then chunk,
// then group, so a wave's groups in one chunk are one contiguous range, and
// hdr is in the same order: off / 16 | (bytes / 16) << 40.
// tile[rb * nch + ch] = tk0 | ntk << 16: the lags row block rb uses in chunk ch.
struct Band {
    int64_t rows = 0, cols = 0, nch = 0, nrb = 0, lag0 = 0, lag1 = 0;
    int64_t nnz = 0;        // stored values (lags between a pair's first and last value)
    size_t bytes = 0;       // stream bytes (words, values, alignment)
    int tmax = 0;           // largest staged lag range of a tile
    int lmax = 0;           // longest run of a pair
    int nsplit = 1;         // chunk splits of the product (partial sums)
    int waves = 16;         // waves per work-group
    int np = 1;             // 1 KB copy pieces per batch (two batch buffers a wave)
    int block = 1;          // steps of one pass (products per value); 1: one step
    int64_t cmax = 0;       // most chunks holding values in one row block
    bool direct = false;    // a one-step band (block 1): stored as row lists, the row product
    DBuf hdr, tile, stream;
    DBuf clist, clen;       // clist[rb][j], j < clen[rb]: the chunks of row block rb that hold values
    // row lists (direct bands): row r holds entries rptr[r] .. rptr[r + 1] - 1,
    // each a value (FP32 or FP64, the group stream's) and col << 4 | k, in
    // column then lag order; the group stream is freed
    DBuf rptr, rval, rcode;
};

// Build a family from dense FP64 lag matrices, rows and columns in the
// stored orders rp, cp (stored index -> matrix index): value (k, r, c) is
// srcA[(k - lag0) * lag_stride + rp[r] * row_stride + cp[c]] for r < split and
// srcB[(k - lag0) * lag_stride + rp[r - split] * row_stride + cp[c]] otherwise.
// fp32: values rounded to FP32 with the rounding carried along each pair's lags
// from lag0.  Only the lags kfirst..lag1 are stored (kfirst < 0: lag0), so the
// bands of two adjacent lag ranges hold exactly the values of the band of both.
// block: the steps of one pass of the product: kBandBlock for lags >=
// kBandBlock, or 1 for a one-step band (lags < 16), which is then rewritten
// as row lists.
void build_band(hipStream_t s, int64_t rows, int64_t cols, int64_t lag0, int64_t lag1, const double *srcA,
                const double *srcB, int64_t split, int64_t lag_stride, int64_t row_stride, const int32_t *rp,
                const int32_t *cp, bool fp32, Band &out, int64_t kfirst = -1, int block = 1);

// block 1: part[split][row] = sum over the split's chunks of sum_k X_k(row, .)
// x_k, x_k the ring slot of lag k: slot0 for k = 0, else (head + k - 1) mod K,
// slots [.][ldx] FP64.  block B > 1 (lags >= B): part[split][b][row] for
// b = 0..B-1, the sum for the step b after the current one, whose lag k is
// the current step's lag k - b (slot (head + k - b - 1) mod K)
void launch_band(hipStream_t s, const Band &b, bool fp32, const double *x, int64_t ldx, int64_t K, int64_t head,
                 int64_t slot0, double *part);

// Morton (Z-curve) order of the edge midpoints (cells = false) or the
// triangle centroids: perm[stored index] = index, inv[index] = stored index
void morton_order(const Mesh &m, bool cells, std::vector<int32_t> &perm, std::vector<int32_t> &inv);

// E, M of the factored history into the two slots of em ([2][ld]), the band
// products in stored order (einv, cinv: index -> stored index):
// E_m = sum_s pac[s][m'] - T0 (ps(c+')/A(c+) - ps(c-')/A(c-)), M_m = sum_s pac[s][ne + m'],
// pac and ps summed with the far partials pacf[s][b], psf[s][b] of a pass of
// nb steps (b: the step within the pass; pacf null: none)
void launch_fac_combine(hipStream_t s, int64_t ne, int64_t nc, const int32_t *cells, const double *area, double T0,
                        const int32_t *einv, const int32_t *cinv, const double *pac, int nsac, const double *ps,
                        int nss, const double *pacf, int nsacf, const double *psf, int nssf, int b, int nb,
                        double *em, int64_t ld);

// out[b][e] = sum over the splits s of part[s][b][e] (e < n, b < nb)
void launch_sum_splits(hipStream_t s, int64_t n, int nsplit, int nb, const double *part, double *out);

// after the solve of step i: sv = Sigma^T y (cells), cslot (stored order) = sv / A
void launch_fac_post_a(hipStream_t s, int64_t nc, const int32_t *tri_edge, const int32_t *tri_sign,
                       const double *area, const int32_t *cinv, const double *y, double *sv, double *cslot);
// j = y + Sigma((1/dt~ - 1) zc - zp / dt~) into jslot (stored order) and
// j_out (if not null); x0 (stored order) = -Sigma zc / dt~, lag 0 of the next step
void launch_fac_post_b(hipStream_t s, int64_t ne, double dtn, const int32_t *cells, const int32_t *einv,
                       const double *y, const double *zc, const double *zp, double *jslot, double *j_out, double *x0);

}  // namespace qhp

struct qhp_ctx::FacState {
    // rows [A_k; C_k] x edges and Sq_k cells x cells: the far lags k >= kBandBlock
    // (passes of kBandBlock steps) and the near lags (A, C: 0.., Sq: 1..kBandBlock - 1)
    qhp::Band ac64, ac32, sq64, sq32;
    qhp::Band ac64n, ac32n, sq64n, sq32n;
    bool has_far = false;              // K >= kBandBlock
    int64_t far_start = 0;             // step whose pass the far partials hold
    bool far_valid = false;            // within one qhp_run / qhp_step call
    qhp::DBuf pem64;                   // [P_E; P_M] [2][ne][ld]
    qhp::DBuf tq64;                    // T_0^{-1} [P_E; P_M] [2][ne][ld], for the inverse solve
    qhp::DBuf eperm, einv, cperm, cinv;  // stored orders of the edges and cells
    qhp::DBuf jx, cq, zy, sv, em, pac, ps, pacf, psf;
    qhp::DBuf pacr, psr;               // the far partials summed over splits: [kBandBlock][2 ne], [kBandBlock][nc]
    int zcur = 0;                      // which half of zy holds L_Sigma^+ Sigma^T y_{i-1}
    int pem_variant = -1, pem_splits = 1;  // of the FP64 [P_E P_M] product (also T_0^{-1} [P_E P_M])
};
