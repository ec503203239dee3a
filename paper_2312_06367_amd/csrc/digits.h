// Int8 digit storage of the lag blocks and history vectors and the batched
// history sum on the int8 matrix cores (QHP_I8X4).
//
// A value v of a row (block) or column (history vector) with scale s =
// max |v| / 127 is held as q = rint(v 2^21 / s), clamped to |q| <= 127 2^21,
// and q = t0 2^21 + t1 2^14 + t2 2^7 + t3 with balanced base-128 digits
// (t0 in [-127, 127], t1..t3 in [-64, 64]); the stored value is s q 2^-21.
// Products of digits are exact in int32, so a lag's contribution is exact up
// to the digit products dropped (weight < 2^-28) and one FP64 scaling.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qhp {

__host__ __device__ inline int64_t i8_rows(int64_t n) { return (n + 15) / 16 * 16; }
// bytes of one stored lag block: digit planes then FP64 row scales
__host__ __device__ inline int64_t i8_block_bytes(int64_t ne, int64_t ld)
{
    return i8_rows(ne) * ld * 4 + i8_rows(ne) * 8;
}
// bytes of one ring slot: digit planes of y^T then FP64 column scales
__host__ __device__ inline int64_t i8_slot_bytes(int64_t nrhs, int64_t ld)
{
    return i8_rows(nrhs) * ld * 4 + i8_rows(nrhs) * 8;
}

// T_k (FP64 rows of stride ldt) + carry -> digits and row scales of one
// block; carry [ne][ne] updated to (T_k + carry) - stored
void launch_i8_quantise(hipStream_t s, int64_t ne, int64_t ld, const double *T, int64_t ldt, double *carry,
                        int8_t *block);
// stored block -> FP64 [ne][ne]
void launch_i8_load(hipStream_t s, int64_t ne, int64_t ld, const int8_t *block, double *T);
// y [ne][nrhs] FP64 -> one ring slot (all of it rewritten)
void launch_i8_store_y(hipStream_t s, int64_t ne, int64_t nrhs, int64_t ld, const double *y, int8_t *slot);
// split count of the int8 history kernel for a variant (-1: the default)
int i8_hist_splits(int64_t ne, int64_t kmax, int64_t nrhs, int variant = -1);
// partial: [nsplit][ne][nrhs] FP64 sums of each split's lags; variant in
// [0, i8_variant_count()) (out of range: the default)
void launch_hist_i8(hipStream_t s, int64_t ne, int64_t ld, int64_t nrhs, int64_t kmax, int nsplit,
                    const int8_t *slabs, const int8_t *ring, int64_t n_slots, int64_t head, double *partial,
                    int variant = -1);
int i8_variant_count();
// rows x right-hand sides per work-group, waves per work-group, steps in
// flight, and whether the pieces go straight from memory into LDS
void i8_variant_desc(int v, int *rows, int *cols, int *waves, int *pf, int *dma);

}  // namespace qhp
