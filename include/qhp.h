/*
 * qhp.h -- C ABI of the MI355X (gfx950) marching-on-in-time solver for the
 * quasi-Helmholtz-projector stabilised time-domain combined field integral
 * equation (qHP TD-CFIE) of Le, Cordel, Andriulli and Cools, arXiv 2312.06367.
 *
 * Units are normalised: c = 1 (time is measured as c*t in metres) and the
 * background impedance eta = 1.  Hence T0 = D (scatterer diameter),
 * kappa = 1/dt and dt~ = dt/D (Sec. II-B, III-A).
 *
 * Conventions for every entry point:
 *   - return value: QHP_OK (0) or a negative QHP_E* code; qhp_last_error()
 *     then holds a message.  A failed call leaves the context in the state it
 *     had before the call, except that a failed qhp_step/qhp_run stops the
 *     march (further steps return QHP_ESTATE until qhp_set_incident).
 *   - host pointers are read or written during the call only; the library
 *     keeps no caller pointer.  Pointers documented as "device" must be device
 *     memory of the context's GPU; the library orders its use on the
 *     context's stream and the call returns when the work is complete.
 *   - the context owns all of its device memory and frees it in qhp_destroy:
 *     hipMalloc / hipFree, or the caller's params.dev_alloc / dev_free hook
 *     when one is given.  All work is issued on params.stream (NULL: null
 *     stream).
 *   - order: create -> mesh -> assemble -> set_incident -> step/run; other
 *     orders return QHP_ESTATE.  set_incident may be repeated (restarts the
 *     march at step 0).  Contexts are not thread-safe.
 *   - dense matrices are row-major.
 */
#ifndef QHP_H
#define QHP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    QHP_OK = 0,
    QHP_EINVAL = -1,    /* bad argument                                       */
    QHP_EMESH = -2,     /* open, non-manifold, inconsistently oriented or
                           disconnected mesh, or a zero-area triangle          */
    QHP_ESTATE = -3,    /* call out of order                                  */
    QHP_ENOMEM = -4,    /* device allocation failed                           */
    QHP_EDEVICE = -5,   /* HIP runtime error                                  */
    QHP_ESINGULAR = -6, /* zero pivot in an LU factorisation                  */
    QHP_ENOCONV = -7,   /* iterative solve did not reach its tolerance        */
    QHP_EUNSTABLE = -8  /* non-finite value in the marching solution, or its
                           growth trip (qhp_set_growth_limit)                  */
};
/* Every call that returns int gives QHP_EINVAL for a null handle (context,
 * batch or perceptron) without touching the device; the destroy calls accept a
 * null handle and do nothing. */

/* storage of the lag blocks T_k, k >= 1, and the history-sum arithmetic
 * (T_0, the solve and the post-processing are always FP64):
 *   QHP_F64    FP64 blocks, FP64 products and sums
 *   QHP_F32    FP32 blocks, FP32 copy of y, FP32 products and sums
 *   QHP_BF16   BF16 blocks with a per-block FP32 scale, FP32 sums; y as FP32
 *              (one right-hand side) or, with several right-hand sides, as
 *              two BF16 terms (hi + mid) on the BF16 matrix cores
 *   QHP_F32A   FP32 blocks, FP64 y, products and sums in FP64 (1, 2, 4 or 8
 *              right-hand sides; qhp_history_sum takes one)
 *   QHP_BF16X2 each block as a BF16 pair T_hi + T_lo (4 bytes per entry), y
 *              as three BF16 terms, the five products of weight >= 2^-16
 *              on the BF16 matrix cores with FP32 sums (two or more
 *              right-hand sides)
 *   QHP_I8X4   each block as four signed 8-bit digits of a 28-bit fixed-point
 *              value per row, T_k(i, j) ~ s_ki (t0 + t1 2^-7 + t2 2^-14 +
 *              t3 2^-21) with the FP64 row scale s_ki = max_j |T_k(i, j) + c|
 *              / 127 (4 bytes per entry); y_{i-k} as four digits per column
 *              with an FP64 column scale; the 13 digit products of weight
 *              >= 2^-28 on the int8 matrix cores with exact int32 sums over
 *              each lag, scaled and summed over lags in FP64 (two or more
 *              right-hand sides, N_E <= 65536)
 *   QHP_FAC64  factored history (Sec. IV-A: T_k = P_E W^E_k + P_M W^M_k,
 *              the cost discussion of Sec. IV-C): no dense blocks; the raw
 *              lag matrices A_k, C_k (edge pairs, lags 0..K) and Sq_k, the
 *              q_0 combination of the scalar-potential shell moments
 *              (triangle pairs, lags 1..K; B_k = -T0 Sigma diag(1/A) Sq_k
 *              diag(1/A) Sigma^T) stored lag-banded: for each pair (row,
 *              column) only its run of lags from the first to the last
 *              nonzero value, 64 pairs (two rows, 32 columns) to a group
 *              whose 64 words give each pair's first lag and run length.
 *              With the difference quotients moved onto the history by
 *              summation by parts, the history sum is
 *                E = sum_k A_k j_{i-k} - A_0 P^Sigma y_{i-1} / dt~
 *                    - T0 Sigma diag(1/A) sum_k Sq_k diag(1/A) Sigma^T y_{i-k},
 *                M = sum_k C_k j_{i-k} - C_0 P^Sigma y_{i-1} / dt~,
 *                sum_k T_k y_{i-k} = P_E E + P_M M
 *              (j the current of eq. post_processing): FP64 values, sums
 *              and P_E, P_M; one right-hand side; assembly needs A_K = C_K = 0
 *              (true when no quadrature point pair is farther apart than
 *              (K - 1) dt) and (K + 1) N_E^2 + K N_C^2 doubles of device
 *              memory for the raw matrices while it runs
 *   QHP_FAC32  the same with FP32 band values (rounding carried along each
 *              pair's lags); P_E, P_M, x, products and sums FP64
 * Reduced-precision blocks are rounded lag by lag with the rounding error of
 * each block carried into the next one (c_k = T_k + c_{k-1} - stored_k), so
 * every prefix sum over lags is within one rounding of the FP64 one. */
enum { QHP_F64 = 0, QHP_F32 = 1, QHP_BF16 = 2, QHP_F32A = 3, QHP_BF16X2 = 4, QHP_I8X4 = 5, QHP_FAC64 = 6,
       QHP_FAC32 = 7, QHP_FP8E4M3 = 8 };
/* QHP_FP8E4M3 (qhp_set_precision from QHP_F64 only; not a qhp_create
 * precision): the blocks' values rounded to FP8 E4M3 (OCP: 3 mantissa bits,
 * exponent bias 7) after scaling each block row to a largest magnitude of
 * 240, with the rounding carried from lag to lag, and kept in FP32 words; the
 * context then marches as QHP_F32A (FP64 y and sums).  It measures what FP8
 * storage does to the march; there is no FP8 history kernel. */

/* per-step solve with T_0 (the paper writes only T_0^{-1}, Sec. IV-B) */
enum {
    QHP_SOLVE_LU = 0,   /* LU with partial pivoting once, two triangular solves per step
                           (factors applied in block-inverse form: 1024-row diagonal
                           blocks inverted, and the off-diagonal blocks multiplied by
                           those inverses, on the first LU step; device memory: n^2
                           doubles plus 2 x 1024^2 per started 1024 rows)            */
    QHP_SOLVE_INV = 1,  /* inverse formed once from that LU, one product per step;
                           with QHP_FAC64 / QHP_FAC32 the product is folded into the
                           history's last one: y_i = T_0^{-1} r_i - T_0^{-1} [P_E P_M]
                           [E; M], with T_0^{-1} [P_E P_M] formed at assembly (2 N_E^2
                           doubles more) and T_0^{-1} r_i for every step by
                           qhp_set_incident (FP64, the same values up to rounding
                           order)                                                  */
    QHP_SOLVE_GMRES = 2 /* restarted GMRES, FP32 Arnoldi inside FP64 residual
                           refinement, started from a warm-start guess (set with
                           qhp_set_gmres after assembly; one right-hand side)     */
};

/* start vector of the iterative solve of step i */
enum {
    QHP_WARM_COLD = 0,   /* zero                                               */
    QHP_WARM_PREV = 1,   /* y_{i-1}                                            */
    QHP_WARM_EXTRAP = 2, /* 2 y_{i-1} - y_{i-2}                                */
    QHP_WARM_QUAD = 3,   /* 3 y_{i-1} - 3 y_{i-2} + y_{i-3}                    */
    QHP_WARM_MLP = 4,    /* the attached perceptron's guess from y_{i-1..i-4}  */
    QHP_WARM_BEST = 5    /* the perceptron's guess or quadratic extrapolation,
                            whichever has the smaller FP64 residual against
                            this step's right-hand side (two residuals per step) */
};

typedef struct qhp_ctx qhp_ctx;

typedef struct {
    double dt;         /* c*dt in metres, > 0                                     */
    double eta_c;      /* coupling of eq. qHP_TDCFIE (the paper's eta^2; 1 here)  */
    int32_t precision; /* QHP_F64 / QHP_F32 / QHP_BF16                             */
    int32_t solver;    /* QHP_SOLVE_LU / QHP_SOLVE_INV (GMRES: qhp_set_gmres)      */
    int32_t n_psi;     /* angular Gauss points per sub-interval; <= 0 means 10    */
    int32_t device;    /* HIP device ordinal                                       */
    void *stream;      /* hipStream_t, or NULL                                     */
    /* Optional device allocator for everything the context, its batches and
     * its perceptron allocate (both NULL: hipMalloc / hipFree; one without
     * the other: QHP_EINVAL).  dev_alloc(bytes, alloc_user) returns device
     * memory of params.device aligned to 256 bytes, or NULL (the call then
     * fails with QHP_ENOMEM); dev_free(ptr, alloc_user) takes back a pointer
     * it returned.  The library waits for the device before each dev_free,
     * as hipFree does.  Both are called from the thread of the entry point
     * that allocates or frees, only inside library calls; alloc_user is
     * passed through untouched. */
    void *(*dev_alloc)(size_t bytes, void *user);
    void (*dev_free)(void *ptr, void *user);
    void *alloc_user;
    /* Temporal basis pairs (h_i, q_i): 0 or 1 = the hat functions h_i and
     * the q_i of Sec. IV-A; 2 = the shifted quadratic Lagrange interpolators
     * of the Remark of Sec. IV-B (on [(m-1) dt, m dt), m = 0..2, the
     * polynomial through the nodes (m-2) dt..m dt, 1 at 0) with q_i' =
     * (h_i - h_{i+1})/dt.  Order 2 adds one lag (K = ceil(D/dt) + 2) and
     * x-weighted shell moments to the assembly; other values: QHP_EINVAL. */
    int32_t temporal_order;
} qhp_params;

/* One incident plane wave (Sec. V); u = t - t0 - k_hat . r
 *   pulse 0: amplitude pol cos(2 pi f0 u) exp(-u^2/(2 sig^2)), sig = 1/(2 pi bw)
 *   pulse 1: (4 amplitude/(w sqrt(pi))) pol exp(-((4/w) u)^2)   (the paper's)
 * f0, bw in cycles per metre of c*t; h_in = k_hat x e_in (eta = 1). */
typedef struct {
    double k_hat[3];
    double pol[3];
    double amplitude;
    double t0;
    int32_t pulse;
    double w;
    double f0;
    double bw;
} qhp_wave;

typedef struct {
    int64_t nv, ne, nc;  /* vertices, edges (= unknowns), triangles          */
    int64_t n_harmonic;  /* 2 - Euler characteristic (global loops)          */
    int64_t K;           /* T_k = 0 for k > K                                */
    int64_t n_rhs;       /* right-hand sides after set_incident              */
    int64_t n_steps;     /* steps with a right-hand side                     */
    int64_t step;        /* steps done since set_incident                    */
    int64_t ld;          /* row stride (elements) of the stored slabs        */
    double diameter;     /* D = largest vertex-vertex distance               */
    size_t slab_bytes;   /* device bytes of the stored T_1..T_K              */
    int64_t hist_variant; /* autotuned history-kernel variant (-1: none)    */
    int64_t hist_splits;  /* lag splits of the history sum                  */
    int64_t raw_nnz;      /* nonzeros of the raw lag matrices A_k, B_k, C_k,
                             k = 1..K (Sec. IV-A): the shell-sparse operands
                             a factored history would stream instead of T_k */
    /* factored history of the precision in use (zeros for dense storage):
       the edge-pair band [A_k; C_k] and the triangle-pair band Sq_k of the
       far lags k >= band_block, applied in passes of band_block steps (one
       pass at the first step of each block of a qhp_run call), and the near
       lags, applied every step; slab_bytes is then the bytes a step streams on
       average: far bands / band_block + near bands + [P_E P_M] */
    size_t band_bytes_pairs, band_bytes_cells;  /* stream bytes (runs, words) */
    int64_t band_nnz_pairs, band_nnz_cells;     /* values stored in the runs  */
    int64_t band_waves_pairs, band_waves_cells; /* waves per work-group of
                                                   their product kernels     */
    int64_t band_pieces_pairs, band_pieces_cells; /* 1 KB copy pieces per
                                                     batch of those kernels  */
    int64_t band_block;                         /* steps of a far pass (0: the
                                                   lags are all near)        */
    size_t band_bytes_near_pairs, band_bytes_near_cells; /* near bands' bytes:
                                                   row lists (values, a 4-byte
                                                   column-and-lag word each,
                                                   row starts)              */
} qhp_info;

/* Create a context (no device work beyond selecting params->device).
 * *out receives the handle; QHP_EINVAL for dt <= 0, an unknown enum or a
 * half-given allocator hook. */
int qhp_create(const qhp_params *params, qhp_ctx **out);

/* Check a surface mesh on the host, with no context and no device: the
 * assumptions of Sec. II-A (closed, connected, orientable Gamma), as
 * qhp_mesh checks them.  Returns QHP_OK, QHP_EINVAL for null or negative
 * sizes, or QHP_EMESH for a triangle index out of range, a repeated vertex in
 * a triangle, an edge not shared by exactly two triangles (open or
 * non-manifold), inconsistently oriented neighbours, a disconnected surface,
 * a zero-area triangle (area below 1e-12 of its longest edge squared, i.e.
 * zero up to rounding), or a vertex whose triangles do not form one disc
 * (non-manifold vertex).  On QHP_OK the optional outputs receive the edge count
 * and the number of global loops N_H = 2 - (N_V - N_E + N_C) (Sec. II-D); if
 * msg is not NULL, msg_len > 0 bytes of it receive the reason (NUL-ended). */
int qhp_check_mesh(const double *xyz, int64_t nv, const int32_t *tri, int64_t nc, int64_t *n_edges,
                   int64_t *n_harmonic, char *msg, int64_t msg_len);

/* Mesh of the scatterer surface Gamma (Sec. II-A: closed, connected,
 * orientable), host arrays: xyz [nv][3] metres, tri [nc][3] vertex indices,
 * counter-clockwise seen from outside.  Builds the edge numbering (edges
 * sorted by (min, max) vertex, oriented min -> max; c+ is the triangle whose
 * vertex cycle runs v- -> v+), Lambda and Sigma (Sec. II-D), the barycentric
 * refinement and the BC coefficients (Sec. II-C).  QHP_EMESH on an invalid
 * mesh. */
int qhp_mesh(qhp_ctx *ctx, const double *xyz, int64_t nv, const int32_t *tri, int64_t nc);

/* Assemble on the GPU: projectors (Sec. II-D, FP64), Gram, Yukawa operators
 * (Sec. II-C), Z~ and X~ (Sec. III-B, III-C), the lag blocks T_0..T_K of eq.
 * dis_TD_CFIE (Sec. IV-A) by semi-analytic quadrature, stores T_1..T_K in the
 * chosen precision and factorises T_0 (FP64 LU).  QHP_ESINGULAR on a zero
 * pivot, QHP_ENOMEM when the slabs do not fit. */
int qhp_assemble(qhp_ctx *ctx);

/* Re-store the assembled T_1..T_K in another precision without assembling
 * again: from QHP_F64 storage (the assembly is FP64) to QHP_F32, QHP_F32A,
 * QHP_BF16, QHP_BF16X2 or QHP_I8X4, freeing the FP64 slabs; between QHP_F32 and
 * QHP_F32A, which share the FP32 storage; or between QHP_FAC64 and QHP_FAC32
 * (a factored assembly keeps both).  Dense and factored storage do not
 * convert into each other (QHP_EINVAL).  Allowed after qhp_assemble; resets
 * the march (call qhp_set_incident again). */
int qhp_set_precision(qhp_ctx *ctx, int32_t precision);

/* Conditioning of the system solved at every step (the study of Sec. V-A,
 * condition number against mesh size and time step), in FP64 on the GPU from
 * the assembled T_0 and the inverse formed from its LU:
 *   *cond1 = |T_0|_1 |T_0^{-1}|_1 (largest absolute column sums, exact);
 *   *cond2 = sigma_max(T_0) / sigma_min(T_0), each largest singular value of
 *            T_0 and T_0^{-1} from power_iters steps of power iteration on
 *            A^T A (a fixed start vector; converged to ~1e-8 after 400
 *            steps on the meshes tried).
 * Either output may be NULL (not computed; not both).  After qhp_assemble;
 * QHP_ESTATE if qhp_release_assembly freed T_0, QHP_EINVAL for
 * power_iters < 1 with cond2 requested. */
int qhp_t0_condition(qhp_ctx *ctx, int32_t power_iters, double *cond1, double *cond2);

/* Switch the per-step T_0 solve (QHP_SOLVE_LU / QHP_SOLVE_INV); both use the
 * FP64 LU of T_0 made by qhp_assemble.  QHP_SOLVE_GMRES keeps the parameters
 * of the last qhp_set_gmres (defaults: tol 1e-10, 40 iterations, 4 inner
 * solves, cold start).  Takes effect at the next step. */
int qhp_set_solver(qhp_ctx *ctx, int32_t solver);

/* Free the FP64 assembly operators that marching no longer needs (Gram,
 * Yukawa and MFIE operators, projectors, preconditioners, raw lag matrices,
 * and the FP64 T_0 and its LU where the chosen solver does not use them),
 * keeping the stored lag blocks, T_0^{-1}, the right-hand sides and the march
 * state: for many scatterers held at once.  Needs qhp_set_incident first;
 * afterwards qhp_set_incident, qhp_set_precision, qhp_get_matrix of a freed
 * operator and switching to a solver whose factors were freed return
 * QHP_ESTATE. */
int qhp_release_assembly(qhp_ctx *ctx);

/* Time the history-sum kernel of every following step with HIP events on
 * the context's stream (enable != 0), or stop.  qhp_hist_time() returns the
 * summed kernel time in ms and the number of timed launches since enabling. */
int qhp_profile(qhp_ctx *ctx, int32_t enable);
int qhp_hist_time(qhp_ctx *ctx, double *ms_total, int64_t *launches);
/* Factored history (QHP_FAC64, QHP_FAC32) while profiling: the summed times
 * (ms, HIP events on the context's stream) of the far passes' banded product
 * over the edge pairs (A_k, C_k) and of the one over the triangle pairs
 * (Sq_k), and the number of passes timed since profiling was enabled (one per
 * qhp_info.band_block steps); zeros for dense storage.  QHP_EINVAL on a null
 * argument. */
int qhp_band_time(qhp_ctx *ctx, double *ms_pairs, double *ms_cells, int64_t *launches);

/* Right-hand sides r_k = -Z~ G^-T e~(t_k) + eta_c X~ G^-1 h(t_k), k = 1..n_steps
 * (Sec. IV-A), for n_rhs waves (host array).  Resets the march to step 0. */
int qhp_set_incident(qhp_ctx *ctx, const qhp_wave *waves, int32_t n_rhs, int32_t n_steps);

/* One marching step (Sec. IV-B): y_i = T_0^{-1}(r_i - sum_{k=1}^{K} T_k y_{i-k})
 * and j_i = P^{LH} y_i + dt~^{-1} P^Sigma (y_i - y_{i-1}) (eq. post_processing).
 * j_out: device [ne][n_rhs] FP64 or NULL.  QHP_EUNSTABLE on a non-finite
 * value or a growth trip; QHP_ESTATE past n_steps. */
int qhp_step(qhp_ctx *ctx, double *j_out);

/* Growth trip of qhp_step / qhp_run: the march stops with QHP_EUNSTABLE when
 * an entry of y_i exceeds limit * max_{k <= i} max |r_k| (the largest
 * right-hand side so far; a stable march keeps |y_i| within a small multiple
 * of it, Sec. V-A).  limit = 0 turns the check off; default 1e8.  QHP_EINVAL
 * for a negative or non-finite limit.  Applies from the next step. */
int qhp_set_growth_limit(qhp_ctx *ctx, double limit);

/* n_steps marching steps.  j_hist / y_hist: device [n_steps][ne][n_rhs] FP64
 * or NULL (step i of the call at index i). */
int qhp_run(qhp_ctx *ctx, int32_t n_steps, double *j_hist, double *y_hist);

int qhp_query(const qhp_ctx *ctx, qhp_info *info);

/* Host arrays: edges [ne][2] = (v-, v+), cells [ne][2] = (c+, c-). */
int qhp_edges(const qhp_ctx *ctx, int32_t *edges, int32_t *cells);

/* Copy an assembled FP64 matrix to host memory out [ne][ne] (parity checks):
 *   which = QHP_MAT_*; k is the lag for the slab and raw lag matrices (raw
 *   lag matrices A_k, B_k, C_k only if qhp_keep_raw(ctx, 1) preceded
 *   qhp_assemble).  Slabs stored in a reduced precision are returned as the
 *   exact values of what is stored. */
enum {
    QHP_MAT_GRAM = 0, QHP_MAT_ZS = 1, QHP_MAT_ZH = 2, QHP_MAT_M = 3,
    QHP_MAT_PSIGMA = 4, QHP_MAT_PLAMBDA = 5, QHP_MAT_PE = 6, QHP_MAT_PM = 7,
    QHP_MAT_SLAB = 8, QHP_MAT_A = 9, QHP_MAT_B = 10, QHP_MAT_C = 11
};
int qhp_get_matrix(const qhp_ctx *ctx, int32_t which, int32_t k, double *out);
int qhp_keep_raw(qhp_ctx *ctx, int32_t keep);

/* The per-step history sum on caller buffers (all device, on `stream`):
 *   b = r - sum_{k=1}^{kmax} T_k y_{i-k}              (Sec. IV-B)
 * slabs: [kmax][ne][ld] in `precision` (T_k at index k-1), ld >= ne a
 *   multiple of 8, columns [ne, ld) ignored; for QHP_BF16X2 ld is a multiple
 *   of 32 and each block holds its hi and lo BF16 planes in matrix-core
 *   operand order, [ceil(ne / 16)][ld / 32][2][512] with entry (i, j) of
 *   plane p at ((i / 16 * ld / 32 + j / 32) * 2 + p) * 512
 *   + (i % 16 + 16 * (j % 32 / 8)) * 8 + j % 8, rows >= ne and columns >= ne
 *   zero; for QHP_I8X4 ld is a multiple of 64 and each block is
 *   R * ld * 4 bytes of digit planes followed by R FP64 row scales
 *   (R = ne rounded up to 16): digit a (0..3, t0 first) of entry (i, j) is
 *   the byte ((i / 16 * ld / 64 + j / 64) * 4 + a) * 1024
 *   + (i % 16 + 16 * (j % 64 / 16)) * 16 + j % 16, digits of rows >= ne and
 *   columns >= ne zero, t0 in [-127, 127], t1..t3 in [-64, 64];
 *   scales: [kmax] FP32 per-slab factors for QHP_BF16 (T_k = scale *
 *   stored), else NULL;
 * ring: y_{i-k} is slot (head + k - 1) mod n_slots, n_slots >= kmax; a slot
 *   is [ld][nrhs] FP64 for QHP_F64 and QHP_F32A, [ld][nrhs] FP32 for QHP_F32
 *   and for QHP_BF16 with nrhs = 1, and for QHP_BF16 with nrhs > 1 and for
 *   QHP_BF16X2 (ld a multiple of 32) three BF16 terms y ~ hi + mid + lo, each
 *   the rounding of what the previous ones leave, in the same operand order
 *   with y^T [nrp][ld] as the matrix ([nrp / 16][ld / 32][3][512], nrp = nrhs
 *   rounded up to 16; entries of columns >= ne are ignored, right-hand sides
 *   >= nrhs must be zero; QHP_BF16 reads hi and mid only); for QHP_I8X4 a
 *   slot is P * ld * 4 bytes of digit planes of y^T (P = nrhs rounded up to
 *   16; entry (n, j) placed as entry (i, j) of a block) followed by P FP64
 *   column scales, y(j, n) ~ scale_n (u0 + u1 2^-7 + u2 2^-14 + u3 2^-21),
 *   digits of columns j >= ne and of right-hand sides >= nrhs zero;
 * r, b: [ne][nrhs] FP64.  nrhs >= 1 (>= 2 for QHP_BF16X2 and QHP_I8X4, 1 for
 * QHP_F32A).
 * The call allocates and frees a scratch buffer of partial sums (QHP_ENOMEM
 * if it cannot) and returns when the stream has finished the work. */
int qhp_history_sum(void *stream, int32_t precision, int64_t ne, int64_t ld, int64_t nrhs,
                    int64_t kmax, const void *slabs, const float *scales, const void *ring,
                    int64_t n_slots, int64_t head, const double *r, double *b);

/* The same sum with the kernel variant fixed (0 <= variant <
 * qhp_history_variants(precision, nrhs); -1 = the default), for callers that
 * tune or test the variants the march's autotuner chooses from.  Every
 * variant computes the same products; they differ in tiling and scheduling.
 * With one right-hand side (11 variants) every variant also sums each row in
 * the same order, so all of them return identical results; the last two stage
 * the blocks through LDS and need FP32 blocks (QHP_F32, QHP_F32A) with
 * ld % 256 == 0, otherwise variant 2 runs in their place.  QHP_EINVAL for a
 * variant out of range. */
int qhp_history_sum_variant(void *stream, int32_t precision, int64_t ne, int64_t ld, int64_t nrhs,
                            int64_t kmax, const void *slabs, const float *scales, const void *ring,
                            int64_t n_slots, int64_t head, const double *r, double *b, int32_t variant);
/* number of history-kernel variants for a precision and right-hand-side count */
int qhp_history_variants(int32_t precision, int64_t nrhs);

/* The history sum of qhp_history_sum_variant (same arguments, kernels and
 * results) that allocates nothing, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  The partial sums of the lag splits (split count x ne x
 * nrhs FP64 values; the split count is that of qhp_history_sum_variant for
 * the same precision, sizes and variant) go to one fixed device array of
 * QHP_NOALLOC_SCRATCH_MB MiB that each GPU the library runs on holds until
 * the process ends; sizes whose partial sums do not fit return QHP_EINVAL,
 * as do the argument errors of qhp_history_sum_variant.  The call only
 * enqueues work on `stream` (it neither allocates nor synchronises) and
 * returns QHP_EDEVICE if a launch fails; the caller waits for the stream.
 * Every call on one GPU uses that GPU's one array, so calls that can overlap
 * on one GPU (different streams without ordering between them) race; calls
 * ordered on one stream do not. */
#define QHP_NOALLOC_SCRATCH_MB 64
int qhp_history_sum_noalloc(void *stream, int32_t precision, int64_t ne, int64_t ld, int64_t nrhs,
                            int64_t kmax, const void *slabs, const float *scales, const void *ring,
                            int64_t n_slots, int64_t head, const double *r, double *b, int32_t variant);

const char *qhp_last_error(const qhp_ctx *ctx);
void qhp_destroy(qhp_ctx *ctx);

/* ---- many scatterers marched together ---------------------------------
 * The marching scheme of Sec. IV-B applied to n independent scatterers of
 * uneven size at once: every step is one replay of a HIP graph of grouped
 * kernels (history sums of all scatterers over work tiles of (scatterer,
 * row block, lag split), biggest scatterer first, then the T_0 products, the ring
 * updates and the post-processing of all scatterers); the per-scatterer step
 * and ring head live in device memory.
 * qhp_batch_create: ctxs[i] must all have had qhp_set_incident, share the
 *   device, precision (F64, F32 or F32A) and n_rhs (1, 2, 4 or 8); each
 *   continues from its current step.  The T_0 product uses the FP64 inverse.
 *   The batch keeps the context pointers: destroy it before them.  While a
 *   batch holds a context, qhp_set_incident and qhp_set_precision on it return
 *   QHP_ESTATE (they would move the buffers the batch works on); the context
 *   may still march on its own with qhp_step / qhp_run, and the next
 *   qhp_batch_run continues from where it stands.  The tile
 *   shape of the history product is autotuned on the batch's own blocks.
 * qhp_batch_create_variant: the same with the history tile shape fixed to
 *   variant in [0, qhp_batch_variants(precision, n_rhs)); -1 autotunes.
 *   QHP_EINVAL for any other value.
 * qhp_batch_variants: the number of history tile shapes for F32 or F32A
 *   blocks (QHP_F32, QHP_F32A) with n_rhs right-hand sides (1 where there
 *   is no choice, 0 for an unsupported precision or n_rhs).
 * qhp_batch_history_variant: the tile shape the batch uses (-1 for NULL).
 * qhp_batch_run: n_steps steps of every scatterer; j_hists is a host array
 *   of n device pointers [n_steps][ne_i][n_rhs] FP64 (or NULL entries / a NULL
 *   array for no output).  QHP_EUNSTABLE on a non-finite value (the growth
 *   trip of qhp_set_growth_limit applies to the contexts' own steps only).
 * qhp_batch_step_times: the per-step times (ms, HIP events around each graph
 *   replay) of the last run, into host ms[n]. */
typedef struct qhp_batch qhp_batch;
int qhp_batch_create(qhp_ctx *const *ctxs, int32_t n, qhp_batch **out);
int qhp_batch_create_variant(qhp_ctx *const *ctxs, int32_t n, int32_t variant, qhp_batch **out);
int qhp_batch_variants(int32_t precision, int32_t n_rhs);
int qhp_batch_history_variant(const qhp_batch *b);
int qhp_batch_run(qhp_batch *b, int32_t n_steps, double *const *j_hists);
int qhp_batch_step_times(const qhp_batch *b, float *ms, int32_t n);
const char *qhp_batch_last_error(const qhp_batch *b);
void qhp_batch_destroy(qhp_batch *b);

/* ---------------------------------------------------------------------------
 * Iterative T_0 solve and learned warm start (an extension: the paper only
 * writes T_0^{-1} in the update of Sec. IV-B).
 *
 * qhp_set_gmres: switch the context's per-step solve to restarted GMRES on
 *   T_0.  The Arnoldi basis and the products with T_0 are FP32 (T_0 rounded
 *   once); each inner solve reduces the FP64 residual r = b - T_0 y by up to
 *   1e-6, and FP64 refinement repeats until |r| <= tol |b| (tol > 0, e.g.
 *   1e-10) or max_refine inner solves of at most m_max (1..512) iterations
 *   each have run; then the step falls back to the LU solve and counts a
 *   fallback.  warm: QHP_WARM_*; QHP_WARM_MLP and QHP_WARM_BEST need
 *   qhp_attach_mlp first.
 *   Needs an assembled context and one right-hand side (QHP_EINVAL else).
 * qhp_gmres_stats: totals since the last reset (or context creation): steps
 *   solved, inner iterations (products with T_0), maximum per step, inner
 *   solves, LU fallbacks; and optionally, into host iters[n] / res0[n], the
 *   per-step iteration counts and relative residuals |b - T_0 x0| / |b| of
 *   the start vectors, for the first n steps recorded.
 * qhp_gmres_reset: clear those records. */
typedef struct {
    int64_t steps, iterations, max_iterations, refinements, fallbacks;
    int64_t network_starts; /* QHP_WARM_BEST steps that started from the perceptron */
} qhp_gmres_info;
int qhp_set_gmres(qhp_ctx *ctx, double tol, int32_t m_max, int32_t max_refine, int32_t warm);
int qhp_gmres_stats(const qhp_ctx *ctx, qhp_gmres_info *info, int32_t *iters, float *res0, int64_t n);
int qhp_gmres_reset(qhp_ctx *ctx);

/* The perceptron that predicts y_i from y_{i-1..i-4}.
 * Coordinates (Sec. II-D decomposition of the RWG span): a vector y maps to
 * f = [l (N_V) | s (N_C) | h (N_H)] with s = (Sigma^T Sigma)^+ Sigma^T y,
 * l = (Lambda^T Lambda)^+ Lambda^T y and h = H^T y, H an orthonormal basis of
 * the harmonic space (built once from the context's projectors; unique up to
 * a rotation); N_F = N_V + N_C + N_H = N_E + 2.  Network, N_in = 4 N_F, on
 * the backward differences d0 = f_{i-1}, d1 = f_{i-1} - f_{i-2},
 * d2 = f_{i-1} - 2 f_{i-2} + f_{i-3}, d3 = f_{i-1} - 3 f_{i-2} + 3 f_{i-3} - f_{i-4}:
 *   x = [d0 / rms(d0), d1 / rms(d1), d2 / rms(d2), d3 / rms(d3)] (0 / 0 = 0),
 *   a1 = tanh(W1 x + b1), a2 = tanh(W2 a1 + b2), o = W3 a2 + b3,
 *   guess f_i = 3 f_{i-1} - 3 f_{i-2} + f_{i-3} + rms(d3) o
 * (o = 0 is quadratic extrapolation).
 * Weights are used as BF16 (products on the matrix cores, FP32 sums), biases
 * and the master copy of every parameter are FP32.  Parameter vector layout
 * (FP32): W1 [H][N_in], b1 [H], W2 [H][H], b2 [H], W3 [N_F][H], b3 [N_F].
 *
 * qhp_mlp_create: for an assembled context (which must outlive it), hidden
 *   width H, Glorot-uniform weights from splitmix64(seed), zero biases, the
 *   output layer scaled by 0.01.
 * qhp_mlp_dims: N_F, parameter count, H.
 * qhp_mlp_set_params / qhp_mlp_get_params: host FP32 [n_params]; setting
 *   also resets the Adam moments.
 * qhp_mlp_features: device y [n][N_E] FP64 -> device f [n][N_F] FP64.
 * qhp_mlp_reconstruct: device f [n][N_F] -> device y [n][N_E] (Lambda l +
 *   Sigma s + H h).
 * qhp_mlp_forward: device x [batch][N_in] FP32 -> device out [batch][N_F]
 *   FP32 (the network output o).
 * qhp_mlp_loss_grad: forward and backward for device x [batch][N_in] and
 *   targets t [batch][N_F] (FP32): loss = mean over batch and outputs of
 *   (o - t)^2 into *loss (host, may be NULL), gradient into host grad
 *   [n_params] (may be NULL; it is also kept for qhp_mlp_adam).
 * qhp_mlp_adam: one Adam step (bias-corrected) with the kept gradient.
 * qhp_mlp_train: features of device y [n_steps][N_E][n_runs] FP64 (the
 *   y_hist layout of qhp_run with n_runs right-hand sides), then `epochs`
 *   passes over every window (run, i >= 4) with rms(d3) > 0, in an order
 *   shuffled from seed, minibatches of `batch`, Adam (lr, 0.9, 0.999, 1e-8)
 *   with targets t = (f_i - 3 f_{i-1} + 3 f_{i-2} - f_{i-3}) / rms(d3);
 *   host epoch_loss[epochs] (may be
 *   NULL) receives each pass's mean minibatch loss.  Device memory:
 *   8 n_steps n_runs N_F bytes of features for the call.
 * qhp_mlp_guess: device f [4][N_F] (rows f_{i-1}, f_{i-2}, f_{i-3}, f_{i-4})
 *   -> device g [N_F], the guess of f_i.
 * qhp_attach_mlp: use m (NULL: none) for QHP_WARM_MLP on ctx.
 * qhp_mlp_destroy: frees m (detaching it from its context). */
typedef struct qhp_mlp qhp_mlp;
int qhp_mlp_create(qhp_ctx *ctx, int32_t hidden, uint64_t seed, qhp_mlp **out);
int qhp_mlp_dims(const qhp_mlp *m, int64_t *n_features, int64_t *n_params, int64_t *hidden);
int qhp_mlp_set_params(qhp_mlp *m, const float *params);
int qhp_mlp_get_params(const qhp_mlp *m, float *params);
int qhp_mlp_features(qhp_mlp *m, const double *y, int64_t n, double *f);
int qhp_mlp_guess(qhp_mlp *m, const double *f, double *g);
int qhp_mlp_reconstruct(qhp_mlp *m, const double *f, int64_t n, double *y);
int qhp_mlp_forward(qhp_mlp *m, const float *x, int32_t batch, float *out);
int qhp_mlp_loss_grad(qhp_mlp *m, const float *x, const float *t, int32_t batch, double *loss, float *grad);
int qhp_mlp_adam(qhp_mlp *m, double lr, double beta1, double beta2, double eps);
int qhp_mlp_train(qhp_mlp *m, const double *y, int64_t n_runs, int64_t n_steps, int32_t epochs, int32_t batch,
                  double lr, uint64_t seed, double *epoch_loss);
int qhp_attach_mlp(qhp_ctx *ctx, qhp_mlp *m);
const char *qhp_mlp_last_error(const qhp_mlp *m);
void qhp_mlp_destroy(qhp_mlp *m);

#ifdef __cplusplus
}
#endif
#endif
