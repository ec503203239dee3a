// Context of the C ABI shared by the library's host sources (not part of the
// ABI): device buffers, error type and the state of one scatterer's march.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <string>
#include <vector>

#include "assembly.h"
#include "qhp_internal.h"

namespace qhp {

struct Fail {
    int code;
    std::string msg;
};

inline void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) throw Fail{e == hipErrorOutOfMemory ? QHP_ENOMEM : QHP_EDEVICE,
                                    std::string(what) + ": " + hipGetErrorString(e)};
}

// Caller-supplied device allocator (qhp_params.dev_alloc / dev_free).  An
// entry point that works for a context makes its allocator current for the
// calling thread (AllocScope); every DBuf allocated meanwhile takes its memory
// from it and remembers it, so the buffer is returned to the same allocator
// whenever it is released.  Without a current allocator: hipMalloc / hipFree.
struct Allocator {
    void *(*alloc)(size_t, void *) = nullptr;
    void (*free)(void *, void *) = nullptr;
    void *user = nullptr;
};
inline thread_local const Allocator *tl_allocator = nullptr;
struct AllocScope {
    const Allocator *prev;
    explicit AllocScope(const Allocator *a) : prev(tl_allocator) { tl_allocator = (a && a->alloc) ? a : nullptr; }
    ~AllocScope() { tl_allocator = prev; }
};

// device allocation owned by a context
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    Allocator owner{};  // where p came from (alloc == nullptr: hipMalloc)
    void alloc(size_t n)
    {
        release();
        if (n == 0) n = 8;
        if (tl_allocator) {
            p = tl_allocator->alloc(n, tl_allocator->user);
            if (!p) throw Fail{QHP_ENOMEM, "caller allocator refused " + std::to_string(n) + " bytes"};
            owner = *tl_allocator;
        } else {
            hipError_t e = hipMalloc(&p, n);
            if (e != hipSuccess) {
                p = nullptr;
                (void)hipGetLastError();
                throw Fail{QHP_ENOMEM, "device allocation of " + std::to_string(n) + " bytes failed"};
            }
            owner = Allocator{};
        }
        bytes = n;
    }
    void release()
    {
        if (p) {
            if (owner.alloc) {
                // hipFree waits for the device; a caller allocator may not, so wait here
                (void)hipDeviceSynchronize();
                owner.free(p, owner.user);
            } else {
                (void)hipFree(p);
            }
        }
        p = nullptr;
        bytes = 0;
        owner = Allocator{};
    }
    void swap(DBuf &o)
    {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(owner, o.owner);
    }
    template <class T>
    T *as() const { return (T *)p; }
    ~DBuf() { release(); }
};

template <class T>
inline void upload(DBuf &b, const std::vector<T> &v, hipStream_t s)
{
    b.alloc(sizeof(T) * std::max<size_t>(v.size(), 1));
    if (!v.empty()) hip_check(hipMemcpyAsync(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s), "upload");
}

inline void zero(DBuf &b, hipStream_t s) { hip_check(hipMemsetAsync(b.p, 0, b.bytes, s), "memset"); }

}  // namespace qhp

struct qhp_mlp;

struct qhp_ctx {
    qhp_params p{};
    qhp::Allocator allocator{};  // from p.dev_alloc / dev_free / alloc_user
    hipStream_t s = nullptr;
    int state = 0;  // 0 created, 1 meshed, 2 assembled, 3 incident set
    std::string err;
    bool keep_raw = false;
    qhp::Mesh mesh;
    int64_t K = 0, ld = 0;
    double T0 = 0, dtn = 0, kappa = 0;
    // device tables
    qhp::DBuf t_xyz, t_tri, t_edges, t_cells, t_tri_edge, t_tri_sign, t_area, t_valence, t_fxyz, t_ftri, t_fparent,
        t_fowner, t_bc_off, t_bc_edge, t_bc_local, t_bc_flux, t_vcell_off, t_vcell_tri, t_vedge_off, t_vedge,
        t_bct_off, t_bct_entry, t_bc_tri;
    qhp::AsmArgs args{};
    // assembled operators (FP64, row-major)
    qhp::DBuf G, Zs, Zh, M, PS, PPL, Pcat, LSp;
    qhp::DBuf slabs, scales_d, T0raw, LU0, ipiv0, perm0, Tinv;
    qhp::DBuf Wsv, Dlsv, Dusv;  // LU factors of T_0 in block-inverse form (first LU step)
    std::vector<float> scales;
    std::vector<std::vector<double>> rawA, rawB, rawC;
    // march state
    int32_t nrhs = 0;
    int64_t n_steps = 0, step = 0, head = 0;
    bool broken = false;
    qhp::DBuf waves_d, rhs, ring64, ring32, ringb, ring8, bvec, zvec, yvec, partial, sv, zc, errflag;
    qhp::DBuf rhst;  // factored history: T_0^{-1} r_i of every step [n_steps][ne] (the inverse solve)
    // FP32 blocks with FP64 y and sums for 2, 4 or 8 right-hand sides: one
    // group of the grouped work-queue kernel (descriptor, device head, counter)
    qhp::DBuf mr_desc, mr_head, mr_counter, ring64t;  // ring64t: [K][nrhs][ld] FP64 copy of the ring
    int64_t mr_tiles = 0, mr_splits = 0;
    int nsplit = 1;
    int64_t raw_nnz = 0;  // nonzeros of A_k, B_k, C_k, k = 1..K
    int hv = -1;  // autotuned variant of the history kernel (single right-hand side, or int8 digits)
    // profiling of the history kernel
    bool profiling = false;
    std::vector<hipEvent_t> ev;
    double hist_ms = 0.0;
    int64_t hist_launches = 0;
    // factored history: events before the edge-pair product, between it and
    // the triangle-pair product, after that (triples); their summed times
    std::vector<hipEvent_t> ev_band;
    double band_ms[2] = {0.0, 0.0};
    int64_t band_launches = 0;
    bool verbose = false;
    std::chrono::steady_clock::time_point t_stage;
    void stage(const char *name)
    {
        if (!verbose) return;
        (void)hipStreamSynchronize(s);
        auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[qhp] %-28s %9.3f s\n", name, std::chrono::duration<double>(now - t_stage).count());
        t_stage = now;
    }
    // iterative T_0 solve (GMRES, FP32 Arnoldi, FP64 refinement) and warm start
    double gm_tol = 1e-10;
    int gm_m = 40, gm_refine = 4, warm = 0;
    qhp::DBuf T0f, gm_V, gm_w, gm_h1, gm_h2, gm_nrm, gm_R, gm_cs, gm_sn, gm_g, gm_inv, gm_y, gm_r, gm_x0;
    double *gm_host = nullptr;  // pinned: residual estimate, |r|^2, |b|^2, the two start residuals
    std::vector<int32_t> gm_iters;
    std::vector<int> gm_pred;  // inner iterations of the last solve per refinement pass
    std::vector<float> gm_res0;
    int64_t gm_refines = 0, gm_fallbacks = 0, gm_net_starts = 0;
    // loop/star/harmonic coordinates of the mesh (learned warm start)
    qhp::DBuf LLp, Hb, ls_sig, ls_lam;
    int64_t ls_nh = -1, ls_cap = 0;
    qhp_mlp *mlp = nullptr;
    bool released = false;  // FP64 assembly operators freed (qhp_release_assembly)
    int batch_refs = 0;     // live batches holding this context (their descriptors point into its buffers)
    // factored history (QHP_FAC64 / QHP_FAC32): the lag-banded raw lag
    // matrices in both value precisions, [P_E; P_M] as two padded blocks
    // [2][ne][ld] (FP64 and FP32), and the march state: the ring of the
    // current j (K slots) plus the lag-0 vector -P^Sigma y_{i-1}/dt~ (slot K),
    // the ring of the cell charges Sigma^T y / A (K slots), L_Sigma^+ Sigma^T y
    // of the last two steps, partial sums, E and M
    struct FacState;
    FacState *fac = nullptr;
    // growth trip of the march: |y_i| > growth_limit * max_{k <= i} max |r_k| (0: off)
    double growth_limit = 1e8;
    qhp::DBuf rpk;  // [n_steps] running maximum of max |r_k|
    qhp::DBuf feat;  // ring of the last four feature vectors [4][nf]
    int64_t feat_n = 0;
    ~qhp_ctx();
};

// make the context's caller allocator (if any) current for this entry point
#define QHP_ALLOC_SCOPE(c) qhp::AllocScope qhp_alloc_scope_((c) ? &(c)->allocator : nullptr)

// record msg as the context's last error and return code
int guard(qhp_ctx *ctx, int code, const std::string &msg);

namespace qhp {
// loop/star/harmonic coordinates of the context's mesh (learned warm start)
void loopstar_prepare(qhp_ctx *c);
void loopstar_features(qhp_ctx *c, const double *Y, int64_t n, int64_t ldy, double *F, int64_t ldf);
void loopstar_reconstruct(qhp_ctx *c, const double *F, int64_t n, int64_t ldf, double *Y, int64_t ldy);
// iterative T_0 solve: buffers, start vector, solve, feature record
void gmres_prepare(qhp_ctx *c);
void warm_start(qhp_ctx *c, const double *b, double *x0);
bool gmres_solve(qhp_ctx *c, const double *b, double *x, int32_t *iters, float *res0);
void warm_record(qhp_ctx *c, const double *y);
}  // namespace qhp
