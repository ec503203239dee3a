// Grouped kernels for marching many scatterers together (descriptor tables,
// device-side step and head counters, graph-capturable).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qhp {

enum { GK_F64 = 0, GK_F32 = 1, GK_F32A = 2 };

// One multi-right-hand-side product group: partial[split][row][rhs] =
// sum over the split's lags k of A_k[row][:] . x_{(head + k) mod n_slots}[:][rhs]
struct GDesc {
    const void *A;          // lag 0 matrix, row stride ld (elements), ld % 8 == 0, columns [cols, ld) zero
    int64_t rows, cols, ld;
    int64_t lag_stride;     // elements between consecutive lag matrices
    int64_t nlags;
    const float *scales;    // per-lag factor or null
    const void *x;          // ring base: slot s at x + s * x_slot_stride, [cols][nrhs]
                            // (or [nrhs][x_ld] when x_ld > 0)
    int64_t x_slot_stride;
    int64_t x_ld;           // row stride of the transposed ring layout, or 0
    int64_t n_slots;
    const int64_t *head;    // device slot of lag 0 (null: 0)
    void *partial;          // [nsplit][rows][nrhs]
    int64_t nsplit;
    int64_t tile0;          // first work tile of this group
    int64_t rowblocks;      // row blocks of grouped_rows_per_tile rows; tiles = rowblocks * nsplit
};

// out[i] = r[step][i] - sum partial (r may be null; negate: + sum)
struct GFin {
    const void *partial;
    int64_t nsplit, n;
    const double *r;
    const int64_t *step;
    double *out;
};

struct GStore {
    const double *y;
    double *ring64;
    float *ring32;
    int64_t slot_stride, n_slots, n;
    const int64_t *head;
    int *err;
    float *ring32t;  // optional transposed FP32 ring [slot][nrhs][ldt]
    int64_t ldt, nrhs;
    double *ring64t;  // optional transposed FP64 ring [slot][nrhs][ldt]
};

struct GPost {
    int64_t ne, nc, nrhs;
    double dtn;
    const int32_t *tri_edge, *tri_sign, *cells;
    const double *ring64;
    int64_t slot_stride, n_slots;
    const int64_t *head, *step;
    double *sv;
    const double *z;
    double *jhist;  // base such that step s writes jhist + s * ne * nrhs (or null)
};

// history tile shapes the batch autotunes over (1 where there is no choice)
int grouped_hist_variants(int kind, int nrhs, bool transposed);
// rows of one work tile of launch_grouped_gemv for this kind, nrhs, ring
// layout and variant
int64_t grouped_rows_per_tile(int kind, int nrhs, bool transposed = false, int variant = 0);
// short description of a history tile shape (for logs)
const char *grouped_variant_name(int kind, int nrhs, bool transposed, int variant);
// whether launch_grouped_gemv of this kind and nrhs reads the ring transposed
bool grouped_ring_transposed(int kind, int nrhs);
// ring [n_slots][ld][nrhs] -> [n_slots][nrhs][ld]
void launch_ring_transpose(hipStream_t s, int64_t n_slots, int64_t ld, int64_t nrhs, const float *in, float *out);
void launch_ring_transpose(hipStream_t s, int64_t n_slots, int64_t ld, int64_t nrhs, const double *in, double *out);
// y [ne][nrhs] FP64 -> one slot [nrhs][ldt] of a transposed ring
void launch_store_transposed(hipStream_t s, int64_t ne, int64_t nrhs, int64_t ldt, const double *y, double *dst);
// transposed: the groups' rings are [nrhs][x_ld] per slot (the batch, for the
// kinds grouped_ring_transposed names) or [cols][nrhs] (one context's own ring)
void launch_grouped_gemv(hipStream_t s, int kind, int nrhs, const GDesc *gd, int ngroups, int64_t total_tiles,
                         unsigned long long *counter, bool transposed, int variant = 0);
void launch_grouped_finish(hipStream_t s, bool acc_double, const GFin *gf, int ngroups, int64_t max_n, int negate);
void launch_grouped_store(hipStream_t s, const GStore *gs, int ngroups, int64_t max_n);
void launch_grouped_post(hipStream_t s, int part, const GPost *gp, int ngroups, int64_t max_n);
void launch_grouped_advance(hipStream_t s, int64_t *steps, int64_t *heads, const int64_t *nslots, int ngroups);
// single-group use of the grouped kernels by one context: *p = v on the stream,
// and b = r - sum of nsplit FP64 partial sums of n entries
void launch_set_i64(hipStream_t s, int64_t *p, int64_t v);
void launch_partial_finish_f64(hipStream_t s, int64_t n, int64_t nsplit, const double *partial, const double *r,
                               double *b);

}  // namespace qhp
