// Launchers of the per-step kernels (history sum, solve, post-processing)
// and of the tested incident fields.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/qhp.h"
#include "digits.h"

namespace qhp {

int hist_splits(int64_t ne, int64_t kmax, int64_t nrhs, int32_t precision);
// rows of one stored lag block (QHP_BF16X2 pads them to whole 16-row tiles)
__host__ __device__ inline int64_t slab_rows(int32_t precision, int64_t ne)
{
    return precision == QHP_BF16X2 ? (ne + 15) / 16 * 16 : ne;
}
// bytes of one stored lag block
__host__ __device__ inline int64_t slab_bytes(int32_t precision, int64_t ne, int64_t ld)
{
    if (precision == QHP_I8X4) return i8_block_bytes(ne, ld);
    const int64_t esz = precision == QHP_F64 ? 8 : (precision == QHP_BF16 ? 2 : 4);
    return esz * slab_rows(precision, ne) * ld;
}
// rows of each BF16 plane of a ring slot for the matrix-core history (nrhs padded to 16)
int64_t ring_bf16_rows(int64_t nrhs);
// y [ne][nrhs] FP64 -> slot planes hi, mid, lo (BF16) in MFMA operand order:
// [nrp / 16][ld / 32][3][512] (see k_hist_mfma)
void launch_store_ybf(hipStream_t s, int64_t ne, int64_t nrhs, int64_t nrp, int64_t ld, const double *y,
                      uint16_t *slot);
// partial: scratch of nsplit * ne * nrhs accumulators (FP64 for QHP_F64,
// QHP_F32A and QHP_I8X4, FP32 otherwise)
void launch_history(hipStream_t s, int32_t precision, int64_t ne, int64_t ld, int64_t nrhs, int64_t kmax,
                    const void *slabs, const float *scales, const void *ring, int64_t n_slots, int64_t head,
                    const double *r, double *b, void *partial, int nsplit, hipEvent_t e0 = nullptr,
                    hipEvent_t e1 = nullptr, int variant = -1);
// argument checks of the caller-buffer history sums (qhp_history_sum*), and
// the lag split count they use (partial sums: split count * ne * nrhs FP64)
bool history_args_valid(int32_t precision, int64_t ne, int64_t ld, int64_t nrhs, int64_t kmax, const void *slabs,
                        const float *scales, const void *ring, int64_t n_slots, int64_t head, const double *r,
                        double *b, int32_t variant);
int history_split_count(int32_t precision, int64_t ne, int64_t nrhs, int64_t kmax, int32_t variant);
int gemv_variant_count();
void gemv_variant_desc(int v, int *rpw, int *unr, int *nt);
void launch_gemv_f64(hipStream_t s, int64_t n, const double *A, const double *x, double *y);
// bound: device pointer to this step's growth bound (the largest |r_k| so
// far), or NULL for no growth check
void launch_store_y(hipStream_t s, int64_t n, const double *y, double *slot64, float *slot32, double *yhist,
                    int *err, const double *bound, double limit);
// out[k] = max over the per entries of step k of |r|
void launch_step_absmax(hipStream_t s, int64_t n_steps, int64_t per, const double *r, double *out);
void launch_post_a(hipStream_t s, int64_t nc, int64_t nrhs, double dtn, const int32_t *tri_edge,
                   const int32_t *tri_sign, const double *y, const double *yprev, double *sv);
void launch_post_b(hipStream_t s, int64_t ne, int64_t nrhs, const int32_t *cells, const double *y, const double *z,
                   double *j);
// lag-carried rounding of T_k (rows of stride ldt) into the stored block [ne][ld]
void launch_quantise_slab(hipStream_t s, int64_t ne, int64_t ld, const double *T, int64_t ldt, double *carry,
                          int32_t precision, float scale, void *out);
// FP32 blocks holding FP8 E4M3 values times a per-row scale (largest |value|
// of the row at 240), lag-carried rounding (carry [ne][ne] FP64)
void launch_quantise_fp8(hipStream_t s, int64_t ne, int64_t ld, const double *T, int64_t ldt, double *carry,
                         double *row_scale, float *out);
void launch_absmax(hipStream_t s, int64_t ne, const double *T, int64_t ldt, const double *carry,
                   unsigned long long *out);
void launch_load_slab(hipStream_t s, int64_t ne, int64_t ld, const void *in, int32_t precision, float scale,
                      double *T);
void launch_exc_local(hipStream_t s, int64_t ntri, const double *xyz, const int32_t *tri, const int32_t *sgn,
                      const qhp_wave *waves, int32_t nrhs, int64_t s0, int64_t ns, double dt, int mode, double *out);
void launch_exc_gather(hipStream_t s, int64_t ne, int64_t nc, int64_t nf, int64_t ncols, const int32_t *cells,
                       const int32_t *tri_edge, const double *eloc, const double *hloc, const int32_t *bct_off,
                       const int32_t *bct_entry, const int32_t *bc_tri, const double *bc_flux, double *EH);
void launch_permute_rhs(hipStream_t s, int64_t ne, int64_t ns, int32_t nrhs, const double *R, double *r);

}  // namespace qhp
