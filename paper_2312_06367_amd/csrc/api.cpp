// C ABI of the qHP TD-CFIE marching solver: context, state machine and the
// orchestration of the gfx950 kernels (see include/qhp.h for the contract).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "assembly.h"
#include "batch.h"
#include "linalg.h"
#include "march.h"
#include "qhp_internal.h"
#include "solve.h"
#include "ctx.h"
#include "factored.h"
#include "temporal.h"

using qhp::DBuf;
using qhp::Fail;
using qhp::hip_check;
using qhp::upload;
using qhp::zero;

namespace {

// Gauss-Legendre nodes on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 1; k < n; ++k) {
                double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

}  // namespace

using qhp::AsmArgs;

int guard(qhp_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

#define API_TRY try {
#define API_CATCH(ctx)                                          \
    }                                                           \
    catch (const Fail &f) { return guard(ctx, f.code, f.msg); } \
    catch (const std::bad_alloc &) { return guard(ctx, QHP_ENOMEM, "host allocation failed"); }

extern "C" int qhp_create(const qhp_params *params, qhp_ctx **out)
{
    if (!params || !out) return QHP_EINVAL;
    if (!(params->dt > 0.0) || params->precision < QHP_F64 || params->precision > QHP_FAC32 ||
        params->temporal_order < 0 || params->temporal_order > 2 ||
        params->solver < QHP_SOLVE_LU || params->solver > QHP_SOLVE_INV || params->n_psi > 32 ||
        (!params->dev_alloc) != (!params->dev_free))
        return QHP_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || params->device < 0 || params->device >= ndev)
        return QHP_EDEVICE;
    qhp_ctx *c = new qhp_ctx();
    c->p = *params;
    if (c->p.n_psi <= 0) c->p.n_psi = 10;
    if (c->p.temporal_order <= 0) c->p.temporal_order = 1;
    if (!(c->p.eta_c > 0.0)) c->p.eta_c = 1.0;
    c->s = (hipStream_t)params->stream;
    c->allocator = qhp::Allocator{params->dev_alloc, params->dev_free, params->alloc_user};
    const char *vb = std::getenv("QHP_VERBOSE");
    c->verbose = vb && vb[0] && vb[0] != '0';
    if (hipSetDevice(params->device) != hipSuccess) {
        delete c;
        return QHP_EDEVICE;
    }
    *out = c;
    return QHP_OK;
}

qhp_ctx::~qhp_ctx()
{
    delete fac;
    if (gm_host) (void)hipHostFree(gm_host);
}

static bool is_fac(int32_t precision) { return precision == QHP_FAC64 || precision == QHP_FAC32; }

extern "C" void qhp_destroy(qhp_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->p.device);
    if (ctx->s) (void)hipStreamSynchronize(ctx->s);
    else (void)hipDeviceSynchronize();
    delete ctx;
}

extern "C" const char *qhp_last_error(const qhp_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" int qhp_check_mesh(const double *xyz, int64_t nv, const int32_t *tri, int64_t nc, int64_t *n_edges,
                              int64_t *n_harmonic, char *msg, int64_t msg_len)
{
    auto say = [&](const std::string &t) {
        if (msg && msg_len > 0) {
            const size_t n = std::min<size_t>(t.size(), (size_t)msg_len - 1);
            std::memcpy(msg, t.data(), n);
            msg[n] = 0;
        }
    };
    if (!xyz || !tri || nv < 0 || nc < 0) {
        say("null or negative argument");
        return QHP_EINVAL;
    }
    try {
        qhp::Mesh m;
        std::string err;
        const int rc = qhp::build_mesh(xyz, nv, tri, nc, m, err);
        if (rc != QHP_OK) {
            say(err);
            return rc;
        }
        for (int64_t v = 0; v < m.nv; ++v)
            if (m.valence[v] > qhp::kMaxValence) {
                say("vertex valence above the supported maximum");
                return QHP_EMESH;
            }
        if (n_edges) *n_edges = m.ne;
        if (n_harmonic) *n_harmonic = m.n_harmonic;
        say("");
        return QHP_OK;
    } catch (const std::bad_alloc &) {
        say("host allocation failed");
        return QHP_ENOMEM;
    }
}

extern "C" int qhp_keep_raw(qhp_ctx *ctx, int32_t keep)
{
    if (!ctx) return QHP_EINVAL;
    ctx->keep_raw = keep != 0;
    return QHP_OK;
}

extern "C" int qhp_mesh(qhp_ctx *ctx, const double *xyz, int64_t nv, const int32_t *tri, int64_t nc)
{
    if (!ctx || !xyz || !tri) return guard(ctx, QHP_EINVAL, "null argument");
    if (ctx->state != 0) return guard(ctx, QHP_ESTATE, "mesh already set");
    API_TRY
    qhp::Mesh m;
    std::string err;
    int rc = qhp::build_mesh(xyz, nv, tri, nc, m, err);
    if (rc != QHP_OK) return guard(ctx, rc, err);
    for (int64_t v = 0; v < m.nv; ++v)
        if (m.valence[v] > qhp::kMaxValence) return guard(ctx, QHP_EMESH, "vertex valence above the supported maximum");
    ctx->mesh = std::move(m);
    ctx->state = 1;
    return QHP_OK;
    API_CATCH(ctx)
}

static void upload_tables(qhp_ctx *c)
{
    const qhp::Mesh &m = c->mesh;
    hipStream_t s = c->s;
    upload(c->t_xyz, m.xyz, s);
    upload(c->t_tri, m.tri, s);
    upload(c->t_edges, m.edges, s);
    upload(c->t_cells, m.cells, s);
    upload(c->t_tri_edge, m.tri_edge, s);
    upload(c->t_tri_sign, m.tri_sign, s);
    upload(c->t_area, m.area, s);
    upload(c->t_valence, m.valence, s);
    upload(c->t_fxyz, m.fxyz, s);
    upload(c->t_ftri, m.ftri, s);
    upload(c->t_fparent, m.fparent, s);
    upload(c->t_fowner, m.fowner, s);
    upload(c->t_bc_off, m.bc_off, s);
    upload(c->t_bc_edge, m.bc_edge, s);
    upload(c->t_bc_local, m.bc_local, s);
    upload(c->t_bc_flux, m.bc_flux, s);
    upload(c->t_vcell_off, m.vcell_off, s);
    upload(c->t_vcell_tri, m.vcell_tri, s);
    upload(c->t_vedge_off, m.vedge_off, s);
    upload(c->t_vedge, m.vedge, s);
    // transposed BC table: entries of each BC function, and entry -> fine triangle
    std::vector<int32_t> cnt(m.ne + 1, 0), bc_tri(m.bc_edge.size());
    for (int64_t t = 0; t < m.nf; ++t)
        for (int32_t e = m.bc_off[t]; e < m.bc_off[t + 1]; ++e) {
            bc_tri[e] = (int32_t)t;
            cnt[m.bc_edge[e] + 1]++;
        }
    for (int64_t i = 0; i < m.ne; ++i) cnt[i + 1] += cnt[i];
    std::vector<int32_t> fillp(cnt.begin(), cnt.end() - 1), ent(m.bc_edge.size());
    for (size_t e = 0; e < m.bc_edge.size(); ++e) ent[fillp[m.bc_edge[e]]++] = (int32_t)e;
    upload(c->t_bct_off, cnt, s);
    upload(c->t_bct_entry, ent, s);
    upload(c->t_bc_tri, bc_tri, s);
    AsmArgs &a = c->args;
    a.nv = m.nv; a.ne = m.ne; a.nc = m.nc; a.nf = m.nf;
    a.xyz = c->t_xyz.as<double>(); a.tri = c->t_tri.as<int32_t>(); a.edges = c->t_edges.as<int32_t>();
    a.cells = c->t_cells.as<int32_t>(); a.tri_edge = c->t_tri_edge.as<int32_t>();
    a.tri_sign = c->t_tri_sign.as<int32_t>(); a.area = c->t_area.as<double>();
    a.valence = c->t_valence.as<int32_t>(); a.fxyz = c->t_fxyz.as<double>(); a.ftri = c->t_ftri.as<int32_t>();
    a.fparent = c->t_fparent.as<int32_t>(); a.fowner = c->t_fowner.as<int32_t>();
    a.bc_off = c->t_bc_off.as<int32_t>(); a.bc_edge = c->t_bc_edge.as<int32_t>();
    a.bc_local = c->t_bc_local.as<int32_t>(); a.bc_flux = c->t_bc_flux.as<double>();
    a.vcell_off = c->t_vcell_off.as<int32_t>(); a.vcell_tri = c->t_vcell_tri.as<int32_t>();
    a.vedge_off = c->t_vedge_off.as<int32_t>(); a.vedge = c->t_vedge.as<int32_t>();
    a.bct_off = c->t_bct_off.as<int32_t>(); a.bct_entry = c->t_bct_entry.as<int32_t>();
    a.bc_tri = c->t_bc_tri.as<int32_t>();
    a.dt = c->p.dt;
    a.coplanar_tol = 1e-12;
    a.ng = c->p.n_psi;
}


// (L + 11^T/n)^{-1} - 11^T/n for the graph Laplacian held (with 1/n added) in L
static void laplacian_pinv(qhp_ctx *c, int64_t n, DBuf &L, DBuf &out)
{
    DBuf piv, info;
    piv.alloc(sizeof(int32_t) * n);
    info.alloc(sizeof(int));
    int rc = qhp::getrf_f64(c->s, n, L.as<double>(), n, piv.as<int32_t>(), info.as<int>());
    if (rc != 0) throw Fail{QHP_ESINGULAR, "graph Laplacian factorisation hit a zero pivot"};
    out.alloc(sizeof(double) * n * n);
    qhp::eye_plus(c->s, n, 1.0, 0.0, L.as<double>(), out.as<double>());
    qhp::getrs_f64(c->s, false, n, n, L.as<double>(), n, piv.as<int32_t>(), out.as<double>(), n);
    qhp::launch_sub_const(c->s, n, out.as<double>());
}

// Store T_k (rows of stride ldt, FP64) into its block in the stored precision
// with lag-carried rounding; returns the per-block scale (BF16: max |T_k + c|).
static float store_lag(hipStream_t s, int64_t ne, int64_t ld, const double *T, int64_t ldt, double *carry,
                       int32_t prec, DBuf &amax, void *out)
{
    float sc = 1.0f;
    if (prec == QHP_I8X4) {
        qhp::launch_i8_quantise(s, ne, ld, T, ldt, carry, (int8_t *)out);
        return sc;
    }
    if (prec == QHP_BF16) {
        unsigned long long bits = 0;
        zero(amax, s);
        qhp::launch_absmax(s, ne, T, ldt, carry, amax.as<unsigned long long>());
        hip_check(hipMemcpyAsync(&bits, amax.p, 8, hipMemcpyDeviceToHost, s), "absmax");
        hip_check(hipStreamSynchronize(s), "absmax");
        double mx;
        std::memcpy(&mx, &bits, 8);
        sc = mx > 0.0 ? (float)mx : 1.0f;
    }
    qhp::launch_quantise_slab(s, ne, ld, T, ldt, prec == QHP_F64 ? nullptr : carry, prec, sc, out);
    return sc;
}

extern "C" int qhp_assemble(qhp_ctx *ctx)
{
    QHP_ALLOC_SCOPE(ctx);
    if (!ctx) return QHP_EINVAL;
    if (ctx->state != 1) return guard(ctx, QHP_ESTATE, ctx->state == 0 ? "no mesh" : "already assembled");
    API_TRY
    qhp_ctx *c = ctx;
    hip_check(hipSetDevice(c->p.device), "hipSetDevice");
    hipStream_t s = c->s;
    const qhp::Mesh &m = c->mesh;
    const int64_t ne = m.ne, nc = m.nc, nv = m.nv;
    const size_t nn = (size_t)ne * ne;
    c->K = qhp::n_lags(m.diameter, c->p.dt, c->p.temporal_order);
    c->T0 = m.diameter;
    c->dtn = c->p.dt / c->T0;
    c->kappa = 1.0 / c->p.dt;
    c->ld = (ne + 511) / 512 * 512;
    const double dtn = c->dtn, kappa = c->kappa;
    c->t_stage = std::chrono::steady_clock::now();
    upload_tables(c);
    {
        std::vector<double> gx, gw;
        gauss_legendre(c->p.n_psi, gx, gw);
        qhp::set_gauss(gx.data(), gw.data(), c->p.n_psi);
    }
    AsmArgs &a = c->args;
    // ---- projectors (Sec. II-D), FP64
    {
        DBuf LS, LL;
        LS.alloc(sizeof(double) * nc * nc);
        LL.alloc(sizeof(double) * nv * nv);
        qhp::launch_laplacians(s, a, LS.as<double>(), LL.as<double>());
        laplacian_pinv(c, nc, LS, c->LSp);
        laplacian_pinv(c, nv, LL, c->LLp);
        c->PS.alloc(sizeof(double) * nn);
        c->PPL.alloc(sizeof(double) * nn);
        qhp::launch_proj(s, ne, a.cells, c->LSp.as<double>(), nc, c->PS.as<double>());
        qhp::launch_proj(s, ne, a.edges, c->LLp.as<double>(), nv, c->PPL.as<double>());
    }
    c->stage("projectors");
    // ---- Gram and Yukawa operators (Sec. II-C)
    c->G.alloc(sizeof(double) * nn);
    zero(c->G, s);
    qhp::launch_gram(s, a, c->G.as<double>());
    c->Zs.alloc(sizeof(double) * nn);
    c->Zh.alloc(sizeof(double) * nn);
    c->M.alloc(sizeof(double) * nn);
    {
        DBuf D;
        D.alloc(sizeof(double) * nv * nv);
        zero(c->Zs, s);
        zero(D, s);
        qhp::launch_yuk_bcbc(s, a, kappa, c->Zs.as<double>(), D.as<double>());
        qhp::symmetrize(s, ne, c->Zs.as<double>());
        qhp::symmetrize(s, nv, D.as<double>());
        qhp::scale_f64(s, ne, ne, -kappa, c->Zs.as<double>(), ne);  // Z^s = -kappa int int g.g G
        qhp::launch_zh(s, a, kappa, D.as<double>(), c->Zh.as<double>());
        zero(c->M, s);
        qhp::launch_yuk_mfie(s, a, kappa, c->M.as<double>());
    }
    hip_check(hipStreamSynchronize(s), "static operators");
    c->stage("gram + yukawa quadrature");
    // ---- Z~ (Sec. III-B), X~ (Sec. III-C), preconditioners
    {
        DBuf left, right, t1, t2, Zt, Xt, Glu, Gpiv, info, Y;
        left.alloc(sizeof(double) * nn);
        right.alloc(sizeof(double) * nn);
        t1.alloc(sizeof(double) * nn);
        t2.alloc(sizeof(double) * nn);
        Zt.alloc(sizeof(double) * nn);
        Xt.alloc(sizeof(double) * nn);
        qhp::eye_plus(s, ne, dtn, 1.0 - dtn, c->PPL.as<double>(), left.as<double>());         // dt~ PP^SH + PP^L
        qhp::eye_plus(s, ne, 1.0, 1.0 / dtn - 1.0, c->PPL.as<double>(), right.as<double>());  // PP^SH + PP^L/dt~
        qhp::gemm_f64(s, false, false, ne, ne, ne, 1.0, c->Zs.as<double>(), ne, right.as<double>(), ne, 0.0, t1.as<double>(), ne);
        qhp::gemm_f64(s, false, false, ne, ne, ne, 1.0, left.as<double>(), ne, t1.as<double>(), ne, 0.0, Zt.as<double>(), ne);
        qhp::gemm_f64(s, false, false, ne, ne, ne, 1.0, c->PPL.as<double>(), ne, c->Zh.as<double>(), ne, 0.0, t2.as<double>(), ne);
        qhp::gemm_f64(s, false, false, ne, ne, ne, 1.0 / dtn, t2.as<double>(), ne, c->PPL.as<double>(), ne, 1.0, Zt.as<double>(), ne);
        qhp::axpby(s, (int64_t)nn, 0.5, c->G.as<double>(), -1.0, c->M.as<double>(), t1.as<double>());  // G/2 - M
        qhp::gemm_f64(s, false, false, ne, ne, ne, 1.0, left.as<double>(), ne, t1.as<double>(), ne, 0.0, Xt.as<double>(), ne);
        // LU of the Gram matrix
        Glu.alloc(sizeof(double) * nn);
        hip_check(hipMemcpyAsync(Glu.p, c->G.p, sizeof(double) * nn, hipMemcpyDeviceToDevice, s), "copy");
        Gpiv.alloc(sizeof(int32_t) * ne);
        info.alloc(sizeof(int));
        if (qhp::getrf_f64(s, ne, Glu.as<double>(), ne, Gpiv.as<int32_t>(), info.as<int>()) != 0)
            throw Fail{QHP_ESINGULAR, "Gram matrix is singular"};
        // P_E = Z~ G^-T (dt~ P^LH + P^Sigma):  Y = G^-1 Z~^T, P_E = Y^T (dt~ I + (1 - dt~) P^Sigma)
        Y.alloc(sizeof(double) * nn);
        qhp::transpose_f64(s, ne, ne, Zt.as<double>(), ne, Y.as<double>(), ne);
        qhp::getrs_f64(s, false, ne, ne, Glu.as<double>(), ne, Gpiv.as<int32_t>(), Y.as<double>(), ne);
        qhp::eye_plus(s, ne, dtn, 1.0 - dtn, c->PS.as<double>(), right.as<double>());
        c->Pcat.alloc(sizeof(double) * nn * 2);
        qhp::gemm_f64(s, true, false, ne, ne, ne, 1.0, Y.as<double>(), ne, right.as<double>(), ne, 0.0,
                      c->Pcat.as<double>(), 2 * ne);
        // P_M = eta_c X~ G^-1:  Y = G^-T X~^T, P_M = eta_c Y^T
        qhp::transpose_f64(s, ne, ne, Xt.as<double>(), ne, Y.as<double>(), ne);
        qhp::getrs_f64(s, true, ne, ne, Glu.as<double>(), ne, Gpiv.as<int32_t>(), Y.as<double>(), ne);
        qhp::transpose_f64(s, ne, ne, Y.as<double>(), ne, t1.as<double>(), ne);
        qhp::scale_f64(s, ne, ne, c->p.eta_c, t1.as<double>(), ne);
        hip_check(hipMemcpy2DAsync(c->Pcat.as<double>() + ne, sizeof(double) * 2 * ne, t1.p, sizeof(double) * ne,
                                   sizeof(double) * ne, ne, hipMemcpyDeviceToDevice, s), "copy P_M");
        hip_check(hipStreamSynchronize(s), "preconditioners");
    }
    c->stage("preconditioners P_E, P_M");
    // ---- lag blocks T_0..T_K (Sec. IV-A) in chunks of lags
    const int64_t K = c->K;
    const int32_t prec = c->p.precision;
    const bool fac = is_fac(prec);
    const size_t blk = fac ? 0 : (size_t)qhp::slab_bytes(prec, ne, c->ld);  // bytes of one stored block
    c->slabs.alloc(fac ? 8 : (size_t)K * blk);
    // factored form: every raw lag matrix kept (FP64, dense) until the bands are built
    qhp::DBuf Afull, Cfull, Sqfull;
    if (fac) {
        Afull.alloc(sizeof(double) * nn * (K + 1));
        Cfull.alloc(sizeof(double) * nn * (K + 1));
        Sqfull.alloc(sizeof(double) * (size_t)nc * nc * K);
    }
    c->scales.assign(K, 1.0f);
    c->T0raw.alloc(sizeof(double) * nn);
    if (c->keep_raw) {
        c->rawA.assign(K + 1, {});
        c->rawB.assign(K + 1, {});
        c->rawC.assign(K + 1, {});
    }
    {
        // temporal order p: shells carry p (V), p + 1 (N) and p + 2 (S)
        // x-weighted moments; lag k combines shells k - p - 1 .. k
        const int ord = c->p.temporal_order, VP = ord, NP = ord + 1, SP = ord + 2;
        const qhp::TemporalBasis tb(ord);
        const size_t nc2 = (size_t)nc * nc;
        const size_t per_shell = sizeof(double) * ((VP + NP) * nn + SP * nc2);
        const size_t budget = (size_t)24 << 30;
        int64_t ch = (int64_t)(budget / per_shell) - (ord + 1);
        ch = std::max<int64_t>(1, std::min<int64_t>(ch, K + 1));
        DBuf V, N, S, Ak, Ck, Ap, Cp, Bk, E, Wst, Tt, amax, Sqk;
        V.alloc(sizeof(double) * nn * VP * (ch + ord + 1));
        N.alloc(sizeof(double) * nn * NP * (ch + ord + 1));
        S.alloc(sizeof(double) * SP * nc2 * (ch + ord + 1));
        if (ord > 1) Sqk.alloc(sizeof(double) * nc2);
        Ak.alloc(sizeof(double) * nn); Ck.alloc(sizeof(double) * nn);
        Ap.alloc(sizeof(double) * nn); Cp.alloc(sizeof(double) * nn);
        Bk.alloc(sizeof(double) * nn); E.alloc(sizeof(double) * nn);
        Wst.alloc(sizeof(double) * nn * 2); Tt.alloc(sizeof(double) * nn);
        amax.alloc(sizeof(unsigned long long));
        DBuf nnz;  // nonzeros of the raw lag matrices, k >= 1
        nnz.alloc(sizeof(unsigned long long));
        zero(nnz, s);
        DBuf carry;  // rounding carried from lag to lag (reduced precisions only)
        if (prec != QHP_F64) {
            carry.alloc(sizeof(double) * nn);
            zero(carry, s);
        }
        zero(Ap, s);
        zero(Cp, s);
        for (int64_t k0 = 0; k0 <= K; k0 += ch) {
            int64_t k1 = std::min<int64_t>(k0 + ch - 1, K);
            int64_t j0 = std::max<int64_t>(k0 - (ord + 1), 0), j1 = std::min<int64_t>(k1, K - 1);
            zero(V, s);
            zero(N, s);
            zero(S, s);
            if (j1 >= j0) {
                qhp::launch_ret_coarse(s, a, ord, j0, j1, V.as<double>(), S.as<double>());
                qhp::launch_ret_bc(s, a, ord, j0, j1, N.as<double>());
                for (int64_t j = j0; j <= j1; ++j) {
                    for (int x = 0; x < VP; ++x) qhp::symmetrize(s, ne, V.as<double>() + ((j - j0) * VP + x) * nn);
                    qhp::launch_sym_s(s, nc, SP, S.as<double>() + (j - j0) * SP * nc2);
                }
            }
            c->stage("retarded shell quadrature");
            // moment x^a of shell j (nullptr outside the chunk's shells)
            auto shellV = [&](int64_t j, int x = 0) -> const double * {
                return (j >= j0 && j <= j1) ? V.as<double>() + ((j - j0) * VP + x) * nn : nullptr;
            };
            auto shellN = [&](int64_t j, int x = 0) -> const double * {
                return (j >= j0 && j <= j1) ? N.as<double>() + ((j - j0) * NP + x) * nn : nullptr;
            };
            auto shellS = [&](int64_t j, int x = 0) -> const double * {
                return (j >= j0 && j <= j1) ? S.as<double>() + ((j - j0) * SP + x) * nc2 : nullptr;
            };
            for (int64_t k = k0; k <= k1; ++k) {
                double *sq_k = fac && k >= 1 ? Sqfull.as<double>() + (k - 1) * nc2 : nullptr;
                if (ord == 1) {  // hat functions: the closed combinations
                    qhp::launch_lag_ac(s, (int64_t)nn, k, c->p.dt, shellV(k), shellV(k - 1), shellN(k),
                                       shellN(k - 1), c->G.as<double>(), Ak.as<double>(), Ck.as<double>());
                    qhp::launch_bk(s, a, shellS(k), shellS(k - 1), shellS(k - 2), c->T0, Bk.as<double>());
                    if (sq_k) qhp::launch_sq(s, nc, shellS(k), shellS(k - 1), shellS(k - 2), sq_k);
                } else {  // the x^a moments of every interval the bases span, with their coefficients
                    qhp::LinTerms tA, tC, tS;
                    for (int m = 0; m <= ord; ++m) {
                        for (int x = 0; x < VP; ++x) tA.add(shellV(k - m, x), -tb.dh[m][x] / c->p.dt);
                        for (int x = 0; x < NP; ++x) tC.add(shellN(k - m, x), tb.mf((int)k, m, x));
                    }
                    for (int m = 0; m <= ord + 1; ++m)
                        for (int x = 0; x < SP; ++x) tS.add(shellS(k - m, x), tb.q[m][x]);
                    qhp::launch_lincomb(s, (int64_t)nn, tA, 0.0, nullptr, Ak.as<double>());
                    qhp::launch_lincomb(s, (int64_t)nn, tC, 0.5, k == 0 ? c->G.as<double>() : nullptr,
                                        Ck.as<double>());
                    qhp::launch_lincomb(s, (int64_t)nc2, tS, 0.0, nullptr, sq_k ? sq_k : Sqk.as<double>());
                    qhp::launch_bk_sq(s, a, sq_k ? sq_k : Sqk.as<double>(), c->T0, Bk.as<double>());
                }
                if (fac) {
                    hip_check(hipMemcpyAsync(Afull.as<double>() + k * nn, Ak.p, sizeof(double) * nn,
                                             hipMemcpyDeviceToDevice, s), "raw A");
                    hip_check(hipMemcpyAsync(Cfull.as<double>() + k * nn, Ck.p, sizeof(double) * nn,
                                             hipMemcpyDeviceToDevice, s), "raw C");
                }
                if (k >= 1)
                    for (const DBuf *m : {&Ak, &Bk, &Ck})
                        qhp::count_nonzero(s, (int64_t)nn, m->as<double>(), nnz.as<unsigned long long>());
                if (c->keep_raw) {
                    c->rawA[k].resize(nn);
                    c->rawB[k].resize(nn);
                    c->rawC[k].resize(nn);
                    hip_check(hipMemcpyAsync(c->rawA[k].data(), Ak.p, sizeof(double) * nn, hipMemcpyDeviceToHost, s), "raw");
                    hip_check(hipMemcpyAsync(c->rawB[k].data(), Bk.p, sizeof(double) * nn, hipMemcpyDeviceToHost, s), "raw");
                    hip_check(hipMemcpyAsync(c->rawC[k].data(), Ck.p, sizeof(double) * nn, hipMemcpyDeviceToHost, s), "raw");
                }
                if (fac && k >= 1) {  // no dense blocks: only T_0 is formed
                    Ap.swap(Ak);
                    Cp.swap(Ck);
                    continue;
                }
                // W^E = A_k + B_k + ((1/dt~ - 1) A_k - A_{k-1}/dt~) P^Sigma (top half of Wst)
                double *WE = Wst.as<double>(), *WM = Wst.as<double>() + nn;
                qhp::axpby(s, (int64_t)nn, 1.0, Ak.as<double>(), 1.0, Bk.as<double>(), WE);
                qhp::axpby(s, (int64_t)nn, 1.0 / dtn - 1.0, Ak.as<double>(), -1.0 / dtn, Ap.as<double>(), E.as<double>());
                qhp::gemm_f64(s, false, false, ne, ne, ne, 1.0, E.as<double>(), ne, c->PS.as<double>(), ne, 1.0, WE, ne);
                // W^M = C_k + ((1/dt~ - 1) C_k - C_{k-1}/dt~) P^Sigma
                hip_check(hipMemcpyAsync(WM, Ck.p, sizeof(double) * nn, hipMemcpyDeviceToDevice, s), "copy");
                qhp::axpby(s, (int64_t)nn, 1.0 / dtn - 1.0, Ck.as<double>(), -1.0 / dtn, Cp.as<double>(), E.as<double>());
                qhp::gemm_f64(s, false, false, ne, ne, ne, 1.0, E.as<double>(), ne, c->PS.as<double>(), ne, 1.0, WM, ne);
                // T_k = [P_E P_M] [W^E; W^M]
                qhp::gemm_f64(s, false, false, ne, ne, 2 * ne, 1.0, c->Pcat.as<double>(), 2 * ne, Wst.as<double>(), ne,
                              0.0, Tt.as<double>(), ne);
                if (k == 0) {
                    hip_check(hipMemcpyAsync(c->T0raw.p, Tt.p, sizeof(double) * nn, hipMemcpyDeviceToDevice, s), "copy");
                } else {
                    c->scales[k - 1] = store_lag(s, ne, c->ld, Tt.as<double>(), ne, carry.as<double>(), prec, amax,
                                                 (char *)c->slabs.p + (size_t)(k - 1) * blk);
                }
                Ap.swap(Ak);
                Cp.swap(Ck);
            }
            hip_check(hipStreamSynchronize(s), "lag blocks");
            c->stage("lag combination + slab GEMMs");
        }
        unsigned long long cnt = 0;
        hip_check(hipMemcpy(&cnt, nnz.p, sizeof(cnt), hipMemcpyDeviceToHost), "nonzero count");
        c->raw_nnz = (int64_t)cnt;
        if (fac) {
            // summation by parts leaves A_K, C_K acting on P^Sigma y_{i-K-1}: they vanish when no
            // quadrature point pair is farther apart than (K - 1) dt, which the bands rely on
            zero(nnz, s);
            qhp::count_nonzero(s, (int64_t)nn, Afull.as<double>() + K * nn, nnz.as<unsigned long long>());
            qhp::count_nonzero(s, (int64_t)nn, Cfull.as<double>() + K * nn, nnz.as<unsigned long long>());
            hip_check(hipMemcpy(&cnt, nnz.p, sizeof(cnt), hipMemcpyDeviceToHost), "nonzero count");
            if (cnt) throw Fail{QHP_EINVAL, "factored history: A_K or C_K is not zero"};
            c->fac = new qhp_ctx::FacState();
            qhp_ctx::FacState &f = *c->fac;
            // edges and cells stored in Morton order of their midpoints / centroids, so that
            // a row block and a column chunk are compact patches with short lag ranges
            std::vector<int32_t> eperm, einv, cperm, cinv;
            qhp::morton_order(m, false, eperm, einv);
            qhp::morton_order(m, true, cperm, cinv);
            upload(f.eperm, eperm, s);
            upload(f.einv, einv, s);
            upload(f.cperm, cperm, s);
            upload(f.cinv, cinv, s);
            // near lags (A, C: 0..B-1; Sq: 1..B-1) applied every step, far lags (B..K) in
            // passes of B steps; the rounding of both is carried from the first lag on,
            // so together they hold exactly the values of one band over all lags
            constexpr int64_t B = qhp::kBandBlock;
            f.has_far = K >= B;
            const int64_t kn = std::min<int64_t>(B - 1, K);
            for (int fp32 = 0; fp32 < 2; ++fp32) {
                qhp::build_band(s, 2 * ne, ne, 0, kn, Afull.as<double>(), Cfull.as<double>(), ne, (int64_t)nn, ne,
                                f.eperm.as<int32_t>(), f.eperm.as<int32_t>(), fp32 != 0, fp32 ? f.ac32n : f.ac64n);
                qhp::build_band(s, nc, nc, 1, kn, Sqfull.as<double>(), Sqfull.as<double>(), nc, nc * nc, nc,
                                f.cperm.as<int32_t>(), f.cperm.as<int32_t>(), fp32 != 0, fp32 ? f.sq32n : f.sq64n);
                if (!f.has_far) continue;
                qhp::build_band(s, 2 * ne, ne, 0, K, Afull.as<double>(), Cfull.as<double>(), ne, (int64_t)nn, ne,
                                f.eperm.as<int32_t>(), f.eperm.as<int32_t>(), fp32 != 0, fp32 ? f.ac32 : f.ac64, B,
                                (int)B);
                qhp::build_band(s, nc, nc, 1, K, Sqfull.as<double>(), Sqfull.as<double>(), nc, nc * nc, nc,
                                f.cperm.as<int32_t>(), f.cperm.as<int32_t>(), fp32 != 0, fp32 ? f.sq32 : f.sq64, B,
                                (int)B);
            }
            // [P_E; P_M] as two padded FP64 blocks
            const int64_t ld = c->ld;
            f.pem64.alloc(sizeof(double) * 2 * ne * ld);
            for (int h = 0; h < 2; ++h)
                qhp::launch_quantise_slab(s, ne, ld, c->Pcat.as<double>() + h * ne, 2 * ne, nullptr, QHP_F64, 1.0f,
                                          f.pem64.as<double>() + h * ne * ld);
            hip_check(hipStreamSynchronize(s), "factored bands");
            if (c->verbose)
                for (const qhp::Band *b : {&f.ac64n, &f.sq64n, &f.ac64, &f.sq64, &f.ac32n, &f.sq32n, &f.ac32, &f.sq32})
                    if (b->rows)
                        std::fprintf(stderr, "[qhp] band %lld x %lld, lags %lld..%lld, passes of %d steps: %.3f GB, "
                                     "%lld values, %d waves, 2 x %d KB a wave, %d lags staged, %d splits\n",
                                     (long long)b->rows, (long long)b->cols, (long long)b->lag0, (long long)b->lag1,
                                     b->block, b->bytes / 1e9, (long long)b->nnz, b->waves, b->np, b->tmax,
                                     b->nsplit);
            c->stage("factored bands");
        }
    }
    upload(c->scales_d, c->scales, s);
    // ---- T_0: FP64 LU, diagonal-block inverses, optional explicit inverse
    {
        c->LU0.alloc(sizeof(double) * nn);
        hip_check(hipMemcpyAsync(c->LU0.p, c->T0raw.p, sizeof(double) * nn, hipMemcpyDeviceToDevice, s), "copy");
        c->ipiv0.alloc(sizeof(int32_t) * ne);
        DBuf info;
        info.alloc(sizeof(int));
        if (qhp::getrf_f64(s, ne, c->LU0.as<double>(), ne, c->ipiv0.as<int32_t>(), info.as<int>()) != 0)
            throw Fail{QHP_ESINGULAR, "T_0 is singular"};
        std::vector<int32_t> ipiv(ne), perm(ne);
        hip_check(hipMemcpy(ipiv.data(), c->ipiv0.p, sizeof(int32_t) * ne, hipMemcpyDeviceToHost), "ipiv");
        for (int64_t i = 0; i < ne; ++i) perm[i] = (int32_t)i;
        for (int64_t j = 0; j < ne; ++j) std::swap(perm[j], perm[ipiv[j]]);
        upload(c->perm0, perm, s);
        // T_0^{-1} from the same LU (used by QHP_SOLVE_INV)
        c->Tinv.alloc(sizeof(double) * nn);
        qhp::eye_plus(s, ne, 1.0, 0.0, c->LU0.as<double>(), c->Tinv.as<double>());
        qhp::getrs_f64(s, false, ne, ne, c->LU0.as<double>(), ne, c->ipiv0.as<int32_t>(), c->Tinv.as<double>(), ne);
        if (c->fac) {  // the inverse solve folded into the factored history's last product
            const int64_t ld = c->ld;
            qhp_ctx::FacState &f = *c->fac;
            f.tq64.alloc(sizeof(double) * 2 * ne * ld);
            zero(f.tq64, s);
            for (int h = 0; h < 2; ++h)
                qhp::gemm_f64(s, false, false, ne, ne, ne, 1.0, c->Tinv.as<double>(), ne,
                              c->Pcat.as<double>() + h * ne, 2 * ne, 0.0, f.tq64.as<double>() + h * ne * ld, ld);
        }
        hip_check(hipStreamSynchronize(s), "T_0 factorisation");
    }
    c->stage("T_0 LU");
    c->state = 2;
    return QHP_OK;
    API_CATCH(ctx)
}

// Pick the fastest history-kernel variant and split count on the context's
// own slabs (timed with HIP events, two launches each after a warm-up).
static int64_t group_splits(int64_t rows, int64_t cols, int64_t nlags);

// descriptor of a context's grouped history (FP32 blocks, FP64 y and sums,
// several right-hand sides, transposed FP64 ring) for tile shape v
static void set_grouped_shape(qhp_ctx *c, int v)
{
    const int64_t ne = c->mesh.ne, K = c->K, ld = c->ld, nr = c->nrhs;
    const int64_t rpt = qhp::grouped_rows_per_tile(qhp::GK_F32A, (int)nr, true, v);
    qhp::GDesc g{};
    g.A = c->slabs.p; g.rows = ne; g.cols = ne; g.ld = ld; g.lag_stride = ne * ld; g.nlags = K;
    g.scales = nullptr;
    g.x = c->ring64t.p; g.x_slot_stride = ld * nr; g.x_ld = ld; g.n_slots = K;
    g.head = c->mr_head.as<int64_t>();
    g.partial = c->partial.p; g.nsplit = group_splits(rpt, ne, K); g.tile0 = 0; g.rowblocks = (ne + rpt - 1) / rpt;
    c->mr_splits = g.nsplit;
    c->mr_tiles = g.rowblocks * g.nsplit;
    c->hv = v;
    hip_check(hipStreamSynchronize(c->s), "descriptor");  // no launch still reads the old one
    hip_check(hipMemcpy(c->mr_desc.p, &g, sizeof(g), hipMemcpyHostToDevice), "descriptor");
}

// the grouped history's tile shape, timed on the context's own blocks
static void autotune_grouped(qhp_ctx *c)
{
    hipStream_t s = c->s;
    const int nv = qhp::grouped_hist_variants(qhp::GK_F32A, (int)c->nrhs, true);
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    qhp::launch_set_i64(s, c->mr_head.as<int64_t>(), 0);
    float best = 1e30f;
    int best_v = 0;
    for (int v = 0; v < nv; ++v) {
        set_grouped_shape(c, v);
        auto run = [&]() {
            qhp::launch_grouped_gemv(s, qhp::GK_F32A, (int)c->nrhs, c->mr_desc.as<qhp::GDesc>(), 1, c->mr_tiles,
                                     c->mr_counter.as<unsigned long long>(), true, v);
        };
        run();
        hip_check(hipEventRecord(e0, s), "event");
        run();
        run();
        hip_check(hipEventRecord(e1, s), "event");
        hip_check(hipEventSynchronize(e1), "event");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
        if (c->verbose)
            std::fprintf(stderr, "[qhp] history, %lld rows per tile (%s): %.3f ms\n",
                         (long long)qhp::grouped_rows_per_tile(qhp::GK_F32A, (int)c->nrhs, true, v),
                         qhp::grouped_variant_name(qhp::GK_F32A, (int)c->nrhs, true, v), ms / 2);
        if (ms < best) {
            best = ms;
            best_v = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    set_grouped_shape(c, best_v);
}

static void autotune_i8(qhp_ctx *c)
{
    hipStream_t s = c->s;
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    float best = 1e30f;
    int best_v = -1, best_s = c->nsplit;
    for (int v = 0; v < qhp::i8_variant_count(); ++v) {
        const int ns = qhp::i8_hist_splits(c->mesh.ne, c->K, c->nrhs, v);
        auto run = [&]() {
            qhp::launch_history(s, QHP_I8X4, c->mesh.ne, c->ld, c->nrhs, c->K, c->slabs.p, nullptr, c->ring8.p, c->K,
                                0, c->rhs.as<double>(), c->bvec.as<double>(), c->partial.p, ns, nullptr, nullptr, v);
        };
        run();
        hip_check(hipEventRecord(e0, s), "event");
        run();
        run();
        hip_check(hipEventRecord(e1, s), "event");
        hip_check(hipEventSynchronize(e1), "event");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
        if (c->verbose) {
            int rows, cols, waves, pf, dma;
            qhp::i8_variant_desc(v, &rows, &cols, &waves, &pf, &dma);
            std::fprintf(stderr, "[qhp] int8 history kernel %d (%d x %d per work-group, %d waves, %d steps in flight%s, "
                         "%d splits): %.3f ms\n", v, rows, cols, waves, pf, dma ? " straight to LDS" : "", ns, ms / 2);
        }
        if (ms < best) {
            best = ms;
            best_v = v;
            best_s = ns;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->hv = best_v;
    c->nsplit = best_s;
}

// the factored history's [P_E P_M] product: the single right-hand-side
// variant and split count (1 or 2) of the dense kernels, timed
static void autotune_fac(qhp_ctx *c)
{
    qhp_ctx::FacState &f = *c->fac;
    hipStream_t s = c->s;
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    float best = 1e30f;
    for (int v = 0; v < qhp::gemv_variant_count(); ++v)
        for (int ns = 1; ns <= 2; ++ns) {
            auto run = [&]() {
                qhp::launch_history(s, QHP_F64, c->mesh.ne, c->ld, 1, 2, f.pem64.p, nullptr, f.em.p, 2, 0,
                                    c->rhs.as<double>(), c->bvec.as<double>(), c->partial.p, ns, nullptr, nullptr, v);
            };
            run();
            hip_check(hipEventRecord(e0, s), "event");
            run();
            run();
            hip_check(hipEventRecord(e1, s), "event");
            hip_check(hipEventSynchronize(e1), "event");
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
            if (ms < best) {
                best = ms;
                f.pem_variant = v;
                f.pem_splits = ns;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->hv = f.pem_variant;
    c->nsplit = f.pem_splits;
    if (c->verbose)
        std::fprintf(stderr, "[qhp] factored history: [P_E P_M] product variant %d, %d splits, %.3f ms\n",
                     f.pem_variant, f.pem_splits, best / 2);
}

static void autotune(qhp_ctx *c)
{
    c->hv = -1;
    if (is_fac(c->p.precision)) return autotune_fac(c);
    if (c->p.precision == QHP_I8X4) return autotune_i8(c);
    if (c->mr_desc.p) return autotune_grouped(c);
    if (c->nrhs != 1) return;
    hipStream_t s = c->s;
    const int64_t ne = c->mesh.ne, K = c->K;
    const int base = c->nsplit;
    int cand[3] = {std::max(1, base / 2), base, (int)std::min<int64_t>(2 * base, K)};
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    const void *ring = c->ring32.p ? c->ring32.p : c->ring64.p;
    const float *sc = c->p.precision == QHP_BF16 ? c->scales_d.as<float>() : nullptr;
    float best = 1e30f;
    int best_v = 2, best_s = base;
    for (int v = 0; v < qhp::gemv_variant_count(); ++v)
        for (int q = 0; q < 3; ++q) {
            if (q > 0 && cand[q] == cand[q - 1]) continue;
            int ns = cand[q];
            qhp::launch_history(s, c->p.precision, ne, c->ld, 1, K, c->slabs.p, sc, ring, K, 0, c->rhs.as<double>(),
                                c->bvec.as<double>(), c->partial.p, ns, nullptr, nullptr, v);
            hip_check(hipEventRecord(e0, s), "event");
            for (int rep = 0; rep < 2; ++rep)
                qhp::launch_history(s, c->p.precision, ne, c->ld, 1, K, c->slabs.p, sc, ring, K, 0,
                                    c->rhs.as<double>(), c->bvec.as<double>(), c->partial.p, ns, nullptr, nullptr, v);
            hip_check(hipEventRecord(e1, s), "event");
            hip_check(hipEventSynchronize(e1), "event");
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
            if (ms < best) {
                best = ms;
                best_v = v;
                best_s = ns;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->hv = best_v;
    c->nsplit = best_s;
    if (c->verbose) {
        int r, u, n;
        qhp::gemv_variant_desc(best_v, &r, &u, &n);
        std::fprintf(stderr, "[qhp] history kernel: %d rows/wave, %d chunks in flight, nt=%d, %d splits, %.3f ms\n", r, u,
                     n, best_s, best / 2);
    }
}

extern "C" int qhp_set_incident(qhp_ctx *ctx, const qhp_wave *waves, int32_t n_rhs, int32_t n_steps)
{
    QHP_ALLOC_SCOPE(ctx);
    if (!ctx) return QHP_EINVAL;
    if (ctx->state < 2) return guard(ctx, QHP_ESTATE, "assemble first");
    if (ctx->released) return guard(ctx, QHP_ESTATE, "assembly operators were released");
    if (ctx->batch_refs > 0) return guard(ctx, QHP_ESTATE, "a live batch holds the context's march buffers");
    if (!waves || n_rhs < 1 || n_steps < 1) return guard(ctx, QHP_EINVAL, "bad waves / n_rhs / n_steps");
    if (ctx->p.precision == QHP_F32A && n_rhs != 1 && n_rhs != 2 && n_rhs != 4 && n_rhs != 8)
        return guard(ctx, QHP_EINVAL, "QHP_F32A takes 1, 2, 4 or 8 right-hand sides");
    if (ctx->p.solver == QHP_SOLVE_GMRES && n_rhs != 1) return guard(ctx, QHP_EINVAL, "GMRES takes one right-hand side");
    if (ctx->p.precision == QHP_BF16X2 && n_rhs < 2)
        return guard(ctx, QHP_EINVAL, "QHP_BF16X2 takes two or more right-hand sides");
    if (ctx->p.precision == QHP_I8X4 && n_rhs < 2)
        return guard(ctx, QHP_EINVAL, "QHP_I8X4 takes two or more right-hand sides");
    if (ctx->p.precision == QHP_I8X4 && ctx->mesh.ne > 65536)
        return guard(ctx, QHP_EINVAL, "QHP_I8X4 takes at most 65536 edges (int32 sums)");
    if (is_fac(ctx->p.precision) && n_rhs != 1)
        return guard(ctx, QHP_EINVAL, "the factored history takes one right-hand side");
    API_TRY
    qhp_ctx *c = ctx;
    hip_check(hipSetDevice(c->p.device), "hipSetDevice");
    hipStream_t s = c->s;
    const qhp::Mesh &m = c->mesh;
    const int64_t ne = m.ne, nc = m.nc, nf = m.nf;
    c->nrhs = n_rhs;
    c->n_steps = n_steps;
    std::vector<qhp_wave> wv(waves, waves + n_rhs);
    upload(c->waves_d, wv, s);
    c->rhs.alloc(sizeof(double) * (size_t)n_steps * ne * n_rhs);
    {
        int64_t ncols_max = std::max<int64_t>(n_rhs, 2048);
        int64_t ns_chunk = std::max<int64_t>(1, ncols_max / n_rhs);
        ns_chunk = std::min<int64_t>(ns_chunk, n_steps);
        int64_t ncols = ns_chunk * n_rhs;
        DBuf eloc, hloc, EH, R, RT;
        eloc.alloc(sizeof(double) * ncols * nc * 3);
        hloc.alloc(sizeof(double) * ncols * nf * 3);
        EH.alloc(sizeof(double) * ncols * 2 * ne);
        R.alloc(sizeof(double) * ncols * ne);
        c->rhst.release();
        if (c->fac) {  // T_0^{-1} r_i of every step, for the inverse solve folded into the history
            c->rhst.alloc(sizeof(double) * (size_t)n_steps * ne * n_rhs);
            RT.alloc(sizeof(double) * ncols * ne);
        }
        for (int64_t s0 = 0; s0 < n_steps; s0 += ns_chunk) {
            int64_t ns = std::min<int64_t>(ns_chunk, n_steps - s0);
            int64_t nco = ns * n_rhs;
            qhp::launch_exc_local(s, nc, c->args.xyz, c->args.tri, c->args.tri_sign, c->waves_d.as<qhp_wave>(),
                                  n_rhs, s0, ns, c->p.dt, 0, eloc.as<double>());
            qhp::launch_exc_local(s, nf, c->args.fxyz, c->args.ftri, nullptr, c->waves_d.as<qhp_wave>(), n_rhs,
                                  s0, ns, c->p.dt, 1, hloc.as<double>());
            qhp::launch_exc_gather(s, ne, nc, nf, nco, c->args.cells, c->args.tri_edge, eloc.as<double>(),
                                   hloc.as<double>(), c->args.bct_off, c->args.bct_entry, c->args.bc_tri,
                                   c->args.bc_flux, EH.as<double>());
            qhp::gemm_f64(s, false, true, nco, ne, 2 * ne, 1.0, EH.as<double>(), 2 * ne, c->Pcat.as<double>(),
                          2 * ne, 0.0, R.as<double>(), ne);
            qhp::launch_permute_rhs(s, ne, ns, n_rhs, R.as<double>(), c->rhs.as<double>() + s0 * ne * n_rhs);
            if (c->rhst.p) {
                qhp::gemm_f64(s, false, true, nco, ne, ne, 1.0, R.as<double>(), ne, c->Tinv.as<double>(), ne, 0.0,
                              RT.as<double>(), ne);
                qhp::launch_permute_rhs(s, ne, ns, n_rhs, RT.as<double>(), c->rhst.as<double>() + s0 * ne * n_rhs);
            }
        }
        // bound of the growth trip: running maximum over the steps of max |r_k|
        std::vector<double> pk(n_steps);
        c->rpk.alloc(sizeof(double) * n_steps);
        qhp::launch_step_absmax(s, n_steps, ne * n_rhs, c->rhs.as<double>(), c->rpk.as<double>());
        hip_check(hipMemcpyAsync(pk.data(), c->rpk.p, sizeof(double) * n_steps, hipMemcpyDeviceToHost, s), "bound");
        hip_check(hipStreamSynchronize(s), "right-hand sides");
        for (int64_t k = 1; k < n_steps; ++k) pk[k] = std::max(pk[k], pk[k - 1]);
        upload(c->rpk, pk, s);
        hip_check(hipStreamSynchronize(s), "right-hand sides");
    }
    const int64_t K = c->K, ld = c->ld;
    c->ring64.alloc(sizeof(double) * K * ld * n_rhs);
    zero(c->ring64, s);
    if (c->p.precision == QHP_F32 || (c->p.precision == QHP_BF16 && n_rhs == 1)) {
        c->ring32.alloc(sizeof(float) * K * ld * n_rhs);
        zero(c->ring32, s);
    }
    c->ringb.release();
    if ((c->p.precision == QHP_BF16 || c->p.precision == QHP_BF16X2) && n_rhs > 1) {
        c->ringb.alloc(sizeof(uint16_t) * K * 3 * qhp::ring_bf16_rows(n_rhs) * ld);
        zero(c->ringb, s);
    }
    c->ring8.release();
    if (c->p.precision == QHP_I8X4) {
        c->ring8.alloc((size_t)K * qhp::i8_slot_bytes(n_rhs, ld));
        zero(c->ring8, s);
    }
    c->bvec.alloc(sizeof(double) * ne * n_rhs);
    c->zvec.alloc(sizeof(double) * ne * n_rhs);
    c->yvec.alloc(sizeof(double) * ne * n_rhs);
    c->nsplit = qhp::hist_splits(ne, K, n_rhs, c->p.precision);
    int64_t max_split = std::min<int64_t>(2 * c->nsplit, K);
    if (c->p.precision == QHP_I8X4)  // every variant the autotuner tries
        for (int v = 0; v < qhp::i8_variant_count(); ++v)
            max_split = std::max<int64_t>(max_split, qhp::i8_hist_splits(ne, K, n_rhs, v));
    const bool grouped = c->p.precision == QHP_F32A && n_rhs > 1;
    if (grouped)  // partial sums for the largest split count of any tile shape
        for (int v = 0; v < qhp::grouped_hist_variants(qhp::GK_F32A, (int)n_rhs, true); ++v)
            max_split = std::max<int64_t>(
                max_split, group_splits(qhp::grouped_rows_per_tile(qhp::GK_F32A, (int)n_rhs, true, v), ne, K));
    c->partial.alloc(sizeof(double) * max_split * ne * n_rhs);
    c->mr_desc.release();
    c->ring64t.release();
    if (grouped) {  // one group of the batch's history kernels on a transposed FP64 ring
        c->mr_head.alloc(sizeof(int64_t));
        c->mr_counter.alloc(sizeof(unsigned long long));
        c->ring64t.alloc(sizeof(double) * K * n_rhs * ld);
        zero(c->ring64t, s);
        c->mr_desc.alloc(sizeof(qhp::GDesc));
        set_grouped_shape(c, 0);
    }
    c->sv.alloc(sizeof(double) * nc * n_rhs);
    c->zc.alloc(sizeof(double) * nc * n_rhs);
    c->errflag.alloc(sizeof(int));
    zero(c->errflag, s);
    if (is_fac(c->p.precision)) {
        qhp_ctx::FacState &f = *c->fac;
        f.jx.alloc(sizeof(double) * (K + 1) * ld);
        f.cq.alloc(sizeof(double) * K * nc);
        f.zy.alloc(sizeof(double) * 2 * nc);
        f.sv.alloc(sizeof(double) * nc);
        f.em.alloc(sizeof(double) * 2 * ld);
        f.pac.alloc(sizeof(double) * std::max(f.ac64n.nsplit, f.ac32n.nsplit) * 2 * ne);
        f.ps.alloc(sizeof(double) * std::max(f.sq64n.nsplit, f.sq32n.nsplit) * nc);
        if (f.has_far) {
            f.pacf.alloc(sizeof(double) * std::max(f.ac64.nsplit, f.ac32.nsplit) * qhp::kBandBlock * 2 * ne);
            f.psf.alloc(sizeof(double) * std::max(f.sq64.nsplit, f.sq32.nsplit) * qhp::kBandBlock * nc);
            f.pacr.alloc(sizeof(double) * qhp::kBandBlock * 2 * ne);
            f.psr.alloc(sizeof(double) * qhp::kBandBlock * nc);
        }
        f.far_valid = false;
        for (qhp::DBuf *b : {&f.jx, &f.cq, &f.zy, &f.em}) zero(*b, s);
        f.zcur = 0;
        if (c->partial.bytes < sizeof(double) * 2 * ne)  // the [P_E P_M] product: at most two splits
            c->partial.alloc(sizeof(double) * 2 * ne);
    }
    hip_check(hipStreamSynchronize(s), "march buffers");
    autotune(c);
    c->step = 0;
    c->head = 0;
    c->feat_n = 0;
    c->broken = false;
    c->state = 3;
    return QHP_OK;
    API_CATCH(ctx)
}

// one marching step; no host synchronisation
static void do_step(qhp_ctx *c, double *j_out, double *y_out)
{
    hipStream_t s = c->s;
    const qhp::Mesh &m = c->mesh;
    const int64_t ne = m.ne, nc = m.nc, nr = c->nrhs, K = c->K, ld = c->ld;
    const int64_t i = c->step + 1;
    const double *r_i = c->rhs.as<double>() + (i - 1) * ne * nr;
    const bool f64 = c->p.precision == QHP_F64;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->profiling) {
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
        c->ev.push_back(e0);
        c->ev.push_back(e1);
    }
    double *y = c->yvec.as<double>();
    bool solved = false;
    if (c->fac) {  // factored history: banded products, E and M, then [P_E P_M]
        qhp_ctx::FacState &f = *c->fac;
        const bool fp32 = c->p.precision == QHP_FAC32;
        const qhp::Band &bac = fp32 ? f.ac32 : f.ac64, &bsq = fp32 ? f.sq32 : f.sq64;
        const qhp::Band &bacn = fp32 ? f.ac32n : f.ac64n, &bsqn = fp32 ? f.sq32n : f.sq64n;
        constexpr int B = qhp::kBandBlock;
        if (e0) hip_check(hipEventRecord(e0, s), "event");
        if (f.has_far && (!f.far_valid || i >= f.far_start + B)) {
            // the far lags of steps i .. i + B - 1 in one pass (ring slots of steps <= i - 1)
            hipEvent_t eb[3] = {nullptr, nullptr, nullptr};
            if (c->profiling)
                for (hipEvent_t &e : eb) {
                    hip_check(hipEventCreate(&e), "event");
                    c->ev_band.push_back(e);
                }
            if (eb[0]) hip_check(hipEventRecord(eb[0], s), "event");
            qhp::launch_band(s, bac, fp32, f.jx.as<double>(), ld, K, c->head, K, f.pacf.as<double>());
            if (eb[1]) hip_check(hipEventRecord(eb[1], s), "event");
            qhp::launch_band(s, bsq, fp32, f.cq.as<double>(), nc, K, c->head, 0, f.psf.as<double>());
            if (eb[2]) hip_check(hipEventRecord(eb[2], s), "event");
            qhp::launch_sum_splits(s, 2 * ne, bac.nsplit, B, f.pacf.as<double>(), f.pacr.as<double>());
            qhp::launch_sum_splits(s, nc, bsq.nsplit, B, f.psf.as<double>(), f.psr.as<double>());
            f.far_start = i;
            f.far_valid = true;
        }
        qhp::launch_band(s, bacn, fp32, f.jx.as<double>(), ld, K, c->head, K, f.pac.as<double>());
        qhp::launch_band(s, bsqn, fp32, f.cq.as<double>(), nc, K, c->head, 0, f.ps.as<double>());
        qhp::launch_fac_combine(s, ne, nc, c->args.cells, c->args.area, c->T0, f.einv.as<int32_t>(),
                                f.cinv.as<int32_t>(), f.pac.as<double>(), bacn.nsplit, f.ps.as<double>(), bsqn.nsplit,
                                f.has_far ? f.pacr.as<double>() : nullptr, 1, f.has_far ? f.psr.as<double>() : nullptr,
                                1, (int)(i - f.far_start), B, f.em.as<double>(), ld);
        // with the inverse solve: y = T_0^{-1} r_i - T_0^{-1} [P_E P_M] [E; M], both factors formed ahead
        solved = c->p.solver == QHP_SOLVE_INV && f.tq64.p && c->rhst.p;
        qhp::launch_history(s, QHP_F64, ne, ld, 1, 2, solved ? f.tq64.p : f.pem64.p, nullptr, f.em.p, 2, 0,
                            solved ? c->rhst.as<double>() + (i - 1) * ne : r_i, solved ? y : c->bvec.as<double>(),
                            c->partial.p, f.pem_splits, nullptr, e1, f.pem_variant);
    } else if (c->mr_desc.p) {  // FP32 blocks, FP64 y and sums, several right-hand sides: the grouped kernel
        qhp::launch_set_i64(s, c->mr_head.as<int64_t>(), c->head);
        if (e0) hip_check(hipEventRecord(e0, s), "event");
        qhp::launch_grouped_gemv(s, qhp::GK_F32A, (int)nr, c->mr_desc.as<qhp::GDesc>(), 1, c->mr_tiles,
                                 c->mr_counter.as<unsigned long long>(), true, c->hv);
        if (e1) hip_check(hipEventRecord(e1, s), "event");
        qhp::launch_partial_finish_f64(s, ne * nr, c->mr_splits, c->partial.as<double>(), r_i, c->bvec.as<double>());
    } else {
        qhp::launch_history(s, c->p.precision, ne, ld, nr, K, c->slabs.p,
                            c->p.precision == QHP_BF16 ? c->scales_d.as<float>() : nullptr,
                            c->ring8.p ? c->ring8.p
                                       : (c->ringb.p ? c->ringb.p : (c->ring32.p ? c->ring32.p : c->ring64.p)),
                            K, c->head, r_i, c->bvec.as<double>(), c->partial.p, c->nsplit, e0, e1, c->hv);
    }
    if (solved) {
        // y came out of the factored history's last product
    } else if (c->p.solver == QHP_SOLVE_GMRES) {
        qhp::warm_start(c, c->bvec.as<double>(), y);
        int32_t it = 0;
        float r0 = 0.f;
        const bool ok = qhp::gmres_solve(c, c->bvec.as<double>(), y, &it, &r0);
        c->gm_iters.push_back(it);
        c->gm_res0.push_back(r0);
        if (!ok) {  // the LU solve decides the step
            c->gm_fallbacks += 1;
            hip_check(hipMemcpyAsync(y, c->bvec.p, sizeof(double) * ne, hipMemcpyDeviceToDevice, s), "copy");
            qhp::getrs_f64(s, false, ne, 1, c->LU0.as<double>(), ne, c->ipiv0.as<int32_t>(), y, 1);
        }
    } else if (c->p.solver == QHP_SOLVE_INV) {
        if (nr == 1) qhp::launch_gemv_f64(s, ne, c->Tinv.as<double>(), c->bvec.as<double>(), y);
        else  // the history's partial sums are consumed: their buffer takes the split-k products
            qhp::gemm_f64_splitk(s, ne, nr, ne, 1.0, c->Tinv.as<double>(), ne, c->bvec.as<double>(), nr, 0.0, y, nr,
                                 c->partial.as<double>(), (int64_t)(c->partial.bytes / sizeof(double)));
    } else {  // LU back-solves, factors in block-inverse form (built on the first LU step)
        if (!c->Wsv.p) {
            c->Wsv.alloc(sizeof(double) * qhp::solve_w_elems(ne));
            c->Dlsv.alloc(sizeof(double) * qhp::solve_d_elems(ne));
            c->Dusv.alloc(sizeof(double) * qhp::solve_d_elems(ne));
            qhp::build_block_solve(s, ne, c->LU0.as<double>(), ne, c->Wsv.as<double>(), c->Dlsv.as<double>(),
                                   c->Dusv.as<double>());
        }
        qhp::launch_block_solve(s, ne, nr, c->Wsv.as<double>(), c->Dlsv.as<double>(), c->Dusv.as<double>(),
                                c->perm0.as<int32_t>(), c->bvec.as<double>(), c->zvec.as<double>(), y,
                                c->partial.as<double>(), (int64_t)(c->partial.bytes / sizeof(double)));
    }
    const int64_t slot = (c->head - 1 + K) % K;
    double *slot64 = c->ring64.as<double>() + slot * ld * nr;
    float *slot32 = c->ring32.p ? c->ring32.as<float>() + slot * ld * nr : nullptr;
    const double *yprev = i > 1 ? c->ring64.as<double>() + c->head * ld * nr : nullptr;
    if (c->fac) {  // j_i and the cell charges into the rings, the lag-0 vector of the next step
        qhp_ctx::FacState &f = *c->fac;
        double *zc = f.zy.as<double>() + (1 - f.zcur) * nc, *zp = f.zy.as<double>() + f.zcur * nc;
        qhp::launch_fac_post_a(s, nc, c->args.tri_edge, c->args.tri_sign, c->args.area, f.cinv.as<int32_t>(), y,
                               f.sv.as<double>(), f.cq.as<double>() + slot * nc);
        qhp::launch_gemv_f64(s, nc, c->LSp.as<double>(), f.sv.as<double>(), zc);
        qhp::launch_fac_post_b(s, ne, c->dtn, c->args.cells, f.einv.as<int32_t>(), y, zc, zp,
                               f.jx.as<double>() + slot * ld, j_out, f.jx.as<double>() + K * ld);
        f.zcur = 1 - f.zcur;
    } else if (j_out) {
        qhp::launch_post_a(s, nc, nr, c->dtn, c->args.tri_edge, c->args.tri_sign, y, yprev, c->sv.as<double>());
        if (nr == 1) qhp::launch_gemv_f64(s, nc, c->LSp.as<double>(), c->sv.as<double>(), c->zc.as<double>());
        else
            qhp::gemm_f64_splitk(s, nc, nr, nc, 1.0, c->LSp.as<double>(), nc, c->sv.as<double>(), nr, 0.0,
                                 c->zc.as<double>(), nr, c->partial.as<double>(),
                                 (int64_t)(c->partial.bytes / sizeof(double)));
        qhp::launch_post_b(s, ne, nr, c->args.cells, y, c->zc.as<double>(), j_out);
    }
    qhp::launch_store_y(s, ne * nr, y, slot64, slot32, y_out, c->errflag.as<int>(), c->rpk.as<double>() + (i - 1),
                        c->growth_limit);
    if (c->ring64t.p) qhp::launch_store_transposed(s, ne, nr, ld, y, c->ring64t.as<double>() + slot * nr * ld);
    if (c->ringb.p) {
        const int64_t nrp = qhp::ring_bf16_rows(nr);
        qhp::launch_store_ybf(s, ne, nr, nrp, ld, y, c->ringb.as<uint16_t>() + slot * 3 * nrp * ld);
    }
    if (c->ring8.p) qhp::launch_i8_store_y(s, ne, nr, ld, y, c->ring8.as<int8_t>() + slot * qhp::i8_slot_bytes(nr, ld));
    if (c->p.solver == QHP_SOLVE_GMRES) qhp::warm_record(c, y);
    c->head = slot;
    c->step = i;
}

static void collect_events(qhp_ctx *c)
{
    for (size_t q = 0; q + 1 < c->ev.size(); q += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev[q], c->ev[q + 1]) == hipSuccess) {
            c->hist_ms += ms;
            c->hist_launches += 1;
        }
    }
    for (auto e : c->ev) (void)hipEventDestroy(e);
    c->ev.clear();
    for (size_t q = 0; q + 2 < c->ev_band.size(); q += 3) {
        float a = 0.f, b = 0.f;
        if (hipEventElapsedTime(&a, c->ev_band[q], c->ev_band[q + 1]) == hipSuccess &&
            hipEventElapsedTime(&b, c->ev_band[q + 1], c->ev_band[q + 2]) == hipSuccess) {
            c->band_ms[0] += a;
            c->band_ms[1] += b;
            c->band_launches += 1;
        }
    }
    for (auto e : c->ev_band) (void)hipEventDestroy(e);
    c->ev_band.clear();
}

static int finish_run(qhp_ctx *c)
{
    hip_check(hipStreamSynchronize(c->s), "march");
    hip_check(hipGetLastError(), "march launch");
    collect_events(c);
    int e = 0;
    hip_check(hipMemcpy(&e, c->errflag.p, sizeof(int), hipMemcpyDeviceToHost), "error flag");
    if (e == 2) {
        c->broken = true;
        return guard(c, QHP_EUNSTABLE, "non-finite value in the marching solution");
    }
    if (e == 3) {
        c->broken = true;
        return guard(c, QHP_EUNSTABLE, "growth trip: |y_i| exceeded the growth limit times the largest |r_k| so far");
    }
    if (e == 1) {
        c->broken = true;
        return guard(c, QHP_EDEVICE, "triangular solve wait exceeded its bound");
    }
    return QHP_OK;
}

extern "C" int qhp_step(qhp_ctx *ctx, double *j_out)
{
    QHP_ALLOC_SCOPE(ctx);
    if (!ctx) return QHP_EINVAL;
    if (ctx->state != 3 || ctx->broken) return guard(ctx, QHP_ESTATE, "set_incident first");
    if (ctx->step >= ctx->n_steps) return guard(ctx, QHP_ESTATE, "no right-hand side left");
    API_TRY
    if (ctx->fac) ctx->fac->far_valid = false;  // far passes live within one call
    do_step(ctx, j_out, nullptr);
    return finish_run(ctx);
    API_CATCH(ctx)
}

extern "C" int qhp_run(qhp_ctx *ctx, int32_t n_steps, double *j_hist, double *y_hist)
{
    QHP_ALLOC_SCOPE(ctx);
    if (!ctx) return QHP_EINVAL;
    if (ctx->state != 3 || ctx->broken) return guard(ctx, QHP_ESTATE, "set_incident first");
    if (n_steps < 0 || ctx->step + n_steps > ctx->n_steps) return guard(ctx, QHP_EINVAL, "past the last right-hand side");
    API_TRY
    const int64_t stride = ctx->mesh.ne * ctx->nrhs;
    if (ctx->fac) ctx->fac->far_valid = false;  // far passes live within one call
    for (int32_t t = 0; t < n_steps; ++t)
        do_step(ctx, j_hist ? j_hist + t * stride : nullptr, y_hist ? y_hist + t * stride : nullptr);
    return finish_run(ctx);
    API_CATCH(ctx)
}

extern "C" int qhp_release_assembly(qhp_ctx *ctx)
{
    if (!ctx) return QHP_EINVAL;
    if (ctx->state != 3) return guard(ctx, QHP_ESTATE, "set_incident first");
    if (ctx->released) return QHP_OK;
    if (hipStreamSynchronize(ctx->s) != hipSuccess) return guard(ctx, QHP_EDEVICE, "synchronise");
    for (DBuf *b : {&ctx->G, &ctx->Zs, &ctx->Zh, &ctx->M, &ctx->PS, &ctx->PPL, &ctx->Pcat, &ctx->LLp})
        b->release();
    if (ctx->p.solver != QHP_SOLVE_GMRES) ctx->T0raw.release();
    if (ctx->p.solver != QHP_SOLVE_LU && ctx->p.solver != QHP_SOLVE_GMRES) {
        ctx->LU0.release();
        ctx->Wsv.release();
        ctx->Dlsv.release();
        ctx->Dusv.release();
    }
    ctx->rawA.clear();
    ctx->rawB.clear();
    ctx->rawC.clear();
    ctx->released = true;
    return QHP_OK;
}

extern "C" int qhp_t0_condition(qhp_ctx *ctx, int32_t power_iters, double *cond1, double *cond2)
{
    QHP_ALLOC_SCOPE(ctx);
    if (!ctx || (!cond1 && !cond2) || (cond2 && power_iters < 1)) return QHP_EINVAL;
    if (ctx->state < 2) return guard(ctx, QHP_ESTATE, "assemble first");
    if (!ctx->T0raw.p || !ctx->Tinv.p) return guard(ctx, QHP_ESTATE, "T_0 or its inverse was released");
    API_TRY
    hipStream_t s = ctx->s;
    const int64_t ne = ctx->mesh.ne;
    const DBuf *mats[2] = {&ctx->T0raw, &ctx->Tinv};
    if (cond1) {
        DBuf partial, colsum;
        partial.alloc(sizeof(double) * qhp::kColChunks * ne);
        colsum.alloc(sizeof(double) * ne);
        std::vector<double> h(ne);
        double norms[2] = {0.0, 0.0};
        for (int q = 0; q < 2; ++q) {
            qhp::launch_col_abs_sums(s, ne, mats[q]->as<double>(), ne, partial.as<double>(), colsum.as<double>());
            hip_check(hipMemcpyAsync(h.data(), colsum.p, sizeof(double) * ne, hipMemcpyDeviceToHost, s), "column sums");
            hip_check(hipStreamSynchronize(s), "column sums");
            for (double v : h) norms[q] = std::max(norms[q], v);
        }
        *cond1 = norms[0] * norms[1];
    }
    if (cond2) {  // sigma_max(T_0) sigma_max(T_0^{-1}) = sigma_max / sigma_min
        DBuf work;
        work.alloc(sizeof(double) * qhp::power_work_elems(ne));
        double sig[2];
        for (int q = 0; q < 2; ++q) {
            sig[q] = qhp::largest_singular_value(s, ne, mats[q]->as<double>(), power_iters, work.as<double>());
            if (!(sig[q] > 0.0)) throw Fail{QHP_EDEVICE, "power iteration failed"};
        }
        *cond2 = sig[0] * sig[1];
    }
    return QHP_OK;
    API_CATCH(ctx)
}

extern "C" int qhp_set_solver(qhp_ctx *ctx, int32_t solver)
{
    if (!ctx) return QHP_EINVAL;
    if (ctx->released && solver == QHP_SOLVE_LU && !ctx->LU0.p)
        return guard(ctx, QHP_ESTATE, "the LU of T_0 was released");
    if (solver == QHP_SOLVE_GMRES) return qhp_set_gmres(ctx, ctx->gm_tol, ctx->gm_m, ctx->gm_refine, ctx->warm);
    if (solver != QHP_SOLVE_LU && solver != QHP_SOLVE_INV) return guard(ctx, QHP_EINVAL, "unknown solver");
    ctx->p.solver = solver;
    return QHP_OK;
}

extern "C" int qhp_set_growth_limit(qhp_ctx *ctx, double limit)
{
    if (!ctx) return QHP_EINVAL;
    if (!(limit >= 0.0) || !std::isfinite(limit)) return guard(ctx, QHP_EINVAL, "growth limit must be finite and >= 0");
    ctx->growth_limit = limit;
    return QHP_OK;
}

extern "C" int qhp_profile(qhp_ctx *ctx, int32_t enable)
{
    if (!ctx) return QHP_EINVAL;
    ctx->profiling = enable != 0;
    ctx->hist_ms = 0.0;
    ctx->hist_launches = 0;
    ctx->band_ms[0] = ctx->band_ms[1] = 0.0;
    ctx->band_launches = 0;
    return QHP_OK;
}

extern "C" int qhp_band_time(qhp_ctx *ctx, double *ms_pairs, double *ms_cells, int64_t *launches)
{
    if (!ctx || !ms_pairs || !ms_cells || !launches) return QHP_EINVAL;
    *ms_pairs = ctx->band_ms[0];
    *ms_cells = ctx->band_ms[1];
    *launches = ctx->band_launches;
    return QHP_OK;
}

extern "C" int qhp_hist_time(qhp_ctx *ctx, double *ms_total, int64_t *launches)
{
    if (!ctx || !ms_total || !launches) return QHP_EINVAL;
    *ms_total = ctx->hist_ms;
    *launches = ctx->hist_launches;
    return QHP_OK;
}

extern "C" int qhp_set_precision(qhp_ctx *ctx, int32_t precision)
{
    QHP_ALLOC_SCOPE(ctx);
    if (!ctx) return QHP_EINVAL;
    if (ctx->state < 2) return guard(ctx, QHP_ESTATE, "assemble first");
    if (ctx->released) return guard(ctx, QHP_ESTATE, "assembly operators were released");
    if (ctx->batch_refs > 0) return guard(ctx, QHP_ESTATE, "a live batch holds the context's blocks");
    if (precision == ctx->p.precision) return QHP_OK;
    if (is_fac(precision) || is_fac(ctx->p.precision)) {
        if (!(is_fac(precision) && is_fac(ctx->p.precision)))
            return guard(ctx, QHP_EINVAL, "dense and factored storage do not convert into each other");
        ctx->p.precision = precision;  // both band precisions are kept
        ctx->state = 2;
        return QHP_OK;
    }
    const bool fp32_pair = (precision == QHP_F32 || precision == QHP_F32A) &&
                           (ctx->p.precision == QHP_F32 || ctx->p.precision == QHP_F32A);
    if (fp32_pair) {  // same FP32 storage, other arithmetic
        ctx->p.precision = precision;
        ctx->ring32.release();
        ctx->ringb.release();
        ctx->ring8.release();
        ctx->state = 2;
        return QHP_OK;
    }
    if (ctx->p.precision != QHP_F64 || (precision != QHP_F32 && precision != QHP_BF16 && precision != QHP_F32A &&
                                        precision != QHP_BF16X2 && precision != QHP_I8X4 && precision != QHP_FP8E4M3))
        return guard(ctx, QHP_EINVAL,
                     "only FP64 slabs can be re-stored, as FP32, BF16, BF16 pairs, int8 digits or FP8 values");
    API_TRY
    if (precision == QHP_FP8E4M3) {  // FP8 values in FP32 words; the march then runs as QHP_F32A
        hipStream_t s = ctx->s;
        const int64_t ne = ctx->mesh.ne, ld = ctx->ld, K = ctx->K;
        const size_t per = (size_t)ne * ld;
        DBuf out, carry, rs;
        out.alloc(sizeof(float) * per * K);
        carry.alloc(sizeof(double) * ne * ne);
        rs.alloc(sizeof(double) * ne);
        zero(carry, s);
        for (int64_t k = 0; k < K; ++k)
            qhp::launch_quantise_fp8(s, ne, ld, ctx->slabs.as<double>() + k * per, ld, carry.as<double>(),
                                     rs.as<double>(), out.as<float>() + k * per);
        hip_check(hipStreamSynchronize(s), "FP8 slabs");
        ctx->slabs.swap(out);
        ctx->scales.assign(K, 1.0f);
        upload(ctx->scales_d, ctx->scales, s);
        ctx->p.precision = QHP_F32A;
        ctx->ring32.release();
        ctx->ringb.release();
        ctx->ring8.release();
        ctx->state = 2;
        return QHP_OK;
    }
    hipStream_t s = ctx->s;
    const int64_t ne = ctx->mesh.ne, ld = ctx->ld, K = ctx->K;
    const size_t per = (size_t)ne * ld;                               // FP64 source block
    const size_t blk = (size_t)qhp::slab_bytes(precision, ne, ld);  // bytes of one stored block
    DBuf out, amax, carry;
    out.alloc(blk * K);
    amax.alloc(sizeof(unsigned long long));
    carry.alloc(sizeof(double) * ne * ne);
    zero(carry, s);
    for (int64_t k = 0; k < K; ++k)
        ctx->scales[k] = store_lag(s, ne, ld, ctx->slabs.as<double>() + k * per, ld, carry.as<double>(), precision, amax,
                                   (char *)out.p + blk * k);
    hip_check(hipStreamSynchronize(s), "convert slabs");
    ctx->slabs.swap(out);
    upload(ctx->scales_d, ctx->scales, s);
    ctx->p.precision = precision;
    ctx->ring32.release();
    ctx->ringb.release();
    ctx->ring8.release();
    ctx->state = 2;
    return QHP_OK;
    API_CATCH(ctx)
}

extern "C" int qhp_query(const qhp_ctx *ctx, qhp_info *info)
{
    if (!ctx || !info) return QHP_EINVAL;
    std::memset(info, 0, sizeof(*info));
    if (ctx->state < 1) return QHP_ESTATE;
    const qhp::Mesh &m = ctx->mesh;
    info->nv = m.nv;
    info->ne = m.ne;
    info->nc = m.nc;
    info->n_harmonic = m.n_harmonic;
    info->diameter = m.diameter;
    info->K = qhp::n_lags(m.diameter, ctx->p.dt, ctx->p.temporal_order);
    info->ld = ctx->ld;
    info->slab_bytes = ctx->slabs.p ? ctx->slabs.bytes : 0;
    if (ctx->fac) {  // the bands and [P_E P_M] of the precision in use
        const bool fp32 = ctx->p.precision == QHP_FAC32;
        const qhp_ctx::FacState &f = *ctx->fac;
        const qhp::Band &ac = fp32 ? f.ac32 : f.ac64, &sq = fp32 ? f.sq32 : f.sq64;
        const qhp::Band &acn = fp32 ? f.ac32n : f.ac64n, &sqn = fp32 ? f.sq32n : f.sq64n;
        // bytes a step streams on average: the far pass once per kBandBlock steps
        info->slab_bytes = (ac.bytes + sq.bytes) / qhp::kBandBlock + acn.bytes + sqn.bytes +
                           (size_t)2 * m.ne * ctx->ld * 8;
        info->band_block = f.has_far ? qhp::kBandBlock : 0;
        info->band_bytes_near_pairs = acn.bytes;
        info->band_bytes_near_cells = sqn.bytes;
        info->band_bytes_pairs = ac.bytes;
        info->band_bytes_cells = sq.bytes;
        info->band_nnz_pairs = ac.nnz;
        info->band_nnz_cells = sq.nnz;
        info->band_waves_pairs = ac.waves;
        info->band_waves_cells = sq.waves;
        info->band_pieces_pairs = ac.np;
        info->band_pieces_cells = sq.np;
    }
    info->n_rhs = ctx->nrhs;
    info->n_steps = ctx->n_steps;
    info->step = ctx->step;
    info->hist_variant = ctx->hv;
    info->hist_splits = ctx->mr_desc.p ? ctx->mr_splits : ctx->nsplit;
    info->raw_nnz = ctx->raw_nnz;
    return QHP_OK;
}

extern "C" int qhp_edges(const qhp_ctx *ctx, int32_t *edges, int32_t *cells)
{
    if (!ctx) return QHP_EINVAL;
    if (ctx->state < 1) return QHP_ESTATE;
    if (edges) std::memcpy(edges, ctx->mesh.edges.data(), sizeof(int32_t) * ctx->mesh.edges.size());
    if (cells) std::memcpy(cells, ctx->mesh.cells.data(), sizeof(int32_t) * ctx->mesh.cells.size());
    return QHP_OK;
}

extern "C" int qhp_get_matrix(const qhp_ctx *cc, int32_t which, int32_t k, double *out)
{
    qhp_ctx *ctx = const_cast<qhp_ctx *>(cc);
    QHP_ALLOC_SCOPE(ctx);
    if (!ctx || !out) return QHP_EINVAL;
    if (ctx->state < 2) return guard(ctx, QHP_ESTATE, "assemble first");
    API_TRY
    const int64_t ne = ctx->mesh.ne;
    const size_t nn = (size_t)ne * ne;
    const DBuf *src = nullptr;
    switch (which) {
    case QHP_MAT_GRAM: src = &ctx->G; break;
    case QHP_MAT_ZS: src = &ctx->Zs; break;
    case QHP_MAT_ZH: src = &ctx->Zh; break;
    case QHP_MAT_M: src = &ctx->M; break;
    case QHP_MAT_PSIGMA: src = &ctx->PS; break;
    case QHP_MAT_PLAMBDA: src = &ctx->PPL; break;
    case QHP_MAT_PE:
    case QHP_MAT_PM: {
        if (!ctx->Pcat.p) return guard(ctx, QHP_ESTATE, "operator released");
        const double *base = ctx->Pcat.as<double>() + (which == QHP_MAT_PM ? ne : 0);
        hip_check(hipMemcpy2D(out, sizeof(double) * ne, base, sizeof(double) * 2 * ne, sizeof(double) * ne, ne,
                              hipMemcpyDeviceToHost), "copy");
        return QHP_OK;
    }
    case QHP_MAT_SLAB: {
        if (k < 0 || k > ctx->K) return guard(ctx, QHP_EINVAL, "lag out of range");
        if (k == 0) { src = &ctx->T0raw; break; }
        if (ctx->fac) return guard(ctx, QHP_ESTATE, "factored storage holds no dense blocks T_k, k >= 1");
        DBuf tmp;
        tmp.alloc(sizeof(double) * nn);
        const int32_t prec = ctx->p.precision;
        const char *blk = (const char *)ctx->slabs.p + (size_t)(k - 1) * qhp::slab_bytes(prec, ne, ctx->ld);
        if (prec == QHP_I8X4) qhp::launch_i8_load(ctx->s, ne, ctx->ld, (const int8_t *)blk, tmp.as<double>());
        else qhp::launch_load_slab(ctx->s, ne, ctx->ld, blk, prec, ctx->scales[k - 1], tmp.as<double>());
        hip_check(hipStreamSynchronize(ctx->s), "dequantise");
        hip_check(hipMemcpy(out, tmp.p, sizeof(double) * nn, hipMemcpyDeviceToHost), "copy");
        return QHP_OK;
    }
    case QHP_MAT_A:
    case QHP_MAT_B:
    case QHP_MAT_C: {
        auto &vv = which == QHP_MAT_A ? ctx->rawA : (which == QHP_MAT_B ? ctx->rawB : ctx->rawC);
        if (k < 0 || k >= (int64_t)vv.size() || vv[k].empty())
            return guard(ctx, QHP_ESTATE, "raw lag matrices not kept (qhp_keep_raw before assemble)");
        std::memcpy(out, vv[k].data(), sizeof(double) * nn);
        return QHP_OK;
    }
    default: return guard(ctx, QHP_EINVAL, "unknown matrix");
    }
    if (!src->p) return guard(ctx, QHP_ESTATE, "operator released");
    hip_check(hipStreamSynchronize(ctx->s), "sync");
    hip_check(hipMemcpy(out, src->p, sizeof(double) * nn, hipMemcpyDeviceToHost), "copy");
    return QHP_OK;
    API_CATCH(ctx)
}

extern "C" int qhp_history_variants(int32_t precision, int64_t nrhs)
{
    if (precision < QHP_F64 || precision > QHP_I8X4 || nrhs < 1) return 0;
    if (precision == QHP_I8X4) return qhp::i8_variant_count();
    return nrhs == 1 ? qhp::gemv_variant_count() : 1;
}

// argument checks shared by the caller-buffer history sums
bool qhp::history_args_valid(int32_t precision, int64_t ne, int64_t ld, int64_t nrhs, int64_t kmax, const void *slabs,
                             const float *scales, const void *ring, int64_t n_slots, int64_t head, const double *r,
                             double *b, int32_t variant)
{
    if (precision < QHP_F64 || precision > QHP_I8X4 || ne < 1 || ld < ne || ld % 8 != 0 || nrhs < 1 || kmax < 0 ||
        (precision == QHP_F32A && nrhs != 1) || (precision == QHP_BF16X2 && (nrhs < 2 || ld % 32 != 0)) ||
        (precision == QHP_I8X4 && (nrhs < 2 || ld % 64 != 0 || ne > 65536)) ||
        (precision == QHP_BF16 && nrhs > 1 && ld % 32 != 0) ||
        n_slots < kmax || head < 0 || (kmax > 0 && (!slabs || !ring)) || !r || !b ||
        variant < -1 || variant >= qhp_history_variants(precision, nrhs))
        return false;
    return !(precision == QHP_BF16 && !scales);
}

int qhp::history_split_count(int32_t precision, int64_t ne, int64_t nrhs, int64_t kmax, int32_t variant)
{
    const int64_t km = std::max<int64_t>(kmax, 1);
    return precision == QHP_I8X4 ? qhp::i8_hist_splits(ne, km, nrhs, variant) : qhp::hist_splits(ne, km, nrhs, precision);
}

extern "C" int qhp_history_sum_variant(void *stream, int32_t precision, int64_t ne, int64_t ld, int64_t nrhs,
                                       int64_t kmax, const void *slabs, const float *scales, const void *ring,
                                       int64_t n_slots, int64_t head, const double *r, double *b, int32_t variant)
{
    if (!qhp::history_args_valid(precision, ne, ld, nrhs, kmax, slabs, scales, ring, n_slots, head, r, b, variant))
        return QHP_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int nsplit = qhp::history_split_count(precision, ne, nrhs, kmax, variant);
    void *partial = nullptr;
    if (hipMalloc(&partial, sizeof(double) * nsplit * ne * nrhs) != hipSuccess) {
        (void)hipGetLastError();
        return QHP_ENOMEM;
    }
    qhp::launch_history(s, precision, ne, ld, nrhs, kmax, slabs, precision == QHP_BF16 ? scales : nullptr, ring,
                        n_slots, head, r, b, partial, nsplit, nullptr, nullptr, variant);
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipGetLastError();
    (void)hipFree(partial);
    return e == hipSuccess ? QHP_OK : QHP_EDEVICE;
}

extern "C" int qhp_history_sum(void *stream, int32_t precision, int64_t ne, int64_t ld, int64_t nrhs, int64_t kmax,
                               const void *slabs, const float *scales, const void *ring, int64_t n_slots, int64_t head,
                               const double *r, double *b)
{
    return qhp_history_sum_variant(stream, precision, ne, ld, nrhs, kmax, slabs, scales, ring, n_slots, head, r, b,
                                   -1);
}

// ------------------------------------------------------------------ batch
// Many scatterers marched together: one graph per step, grouped kernels.
#include "batch.h"

struct qhp_batch {
    std::vector<qhp_ctx *> ctxs;
    hipStream_t s = nullptr;
    int kind = 0, nrhs = 1, n = 0, hv = 0;  // hv: autotuned history tile shape
    bool acc_double = true;
    std::string err;
    DBuf d_hist, d_solve, d_post, f_hist, f_solve, f_post, st, po, steps, heads, nslots, counter, errflag;
    std::vector<DBuf> part_h, part_s, part_p, bvec, yvec, sv, zc, tinv, lsp, ringt;
    int64_t tiles_h = 0, tiles_s = 0, tiles_p = 0, max_ne = 0, max_nc = 0;
    std::vector<qhp::GPost> post_host;
    std::vector<int64_t> synced;  // each context's step when the batch's device state last matched it
    std::vector<qhp_ctx *> held;  // contexts whose batch_refs this batch counts
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<float> step_ms;
    ~qhp_batch()
    {
        for (qhp_ctx *c : held) c->batch_refs -= 1;
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (s) (void)hipStreamDestroy(s);
    }
};

static int bguard(qhp_batch *b, int code, const std::string &msg)
{
    if (b) b->err = msg;
    return code;
}

// split count so that a tile (rows x cols x lags/split) holds ~ 2M elements
static int64_t group_splits(int64_t rows, int64_t cols, int64_t nlags)
{
    const int64_t target = (int64_t)2 << 20;
    int64_t per_lag = rows * cols;
    int64_t lags = std::max<int64_t>(1, target / per_lag);
    int64_t ns = (nlags + lags - 1) / lags;
    return std::max<int64_t>(1, std::min<int64_t>(ns, nlags));
}

// variant: history tile shape, or -1 to autotune it
static void build_batch(qhp_batch *b, int variant)
{
    const int n = b->n;
    hipStream_t s = b->s;
    const qhp_ctx *c0 = b->ctxs[0];
    const int nr = b->nrhs;
    b->part_h.resize(n); b->part_s.resize(n); b->part_p.resize(n); b->bvec.resize(n); b->yvec.resize(n);
    b->sv.resize(n); b->zc.resize(n); b->tinv.resize(n); b->lsp.resize(n); b->ringt.resize(n);
    const bool trans = qhp::grouped_ring_transposed(b->kind, nr);
    // work-queue order: biggest history first
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int x, int y) {
        const qhp_ctx *a = b->ctxs[x], *q = b->ctxs[y];
        return a->K * a->mesh.ne * a->mesh.ne > q->K * q->mesh.ne * q->mesh.ne;
    });
    std::vector<qhp::GDesc> dh(n), ds(n), dp(n), hist_base(n);
    std::vector<qhp::GFin> fh(n), fs(n), fp(n);
    const int nvar = qhp::grouped_hist_variants(b->kind, nr, trans);
    std::vector<qhp::GStore> gs(n);
    b->post_host.assign(n, qhp::GPost{});
    std::vector<int64_t> st0(n), hd0(n), nsl(n);
    const size_t asz = b->acc_double ? 8 : 4;
    int64_t t_h = 0, t_s = 0, t_p = 0;
    b->errflag.alloc(sizeof(int));
    zero(b->errflag, s);
    b->steps.alloc(sizeof(int64_t) * n);
    b->heads.alloc(sizeof(int64_t) * n);
    b->nslots.alloc(sizeof(int64_t) * n);
    for (int q = 0; q < n; ++q) {
        const int i = order[q];
        qhp_ctx *c = b->ctxs[i];
        const int64_t ne = c->mesh.ne, nc = c->mesh.nc, K = c->K, ld = c->ld;
        b->max_ne = std::max(b->max_ne, ne * nr);
        b->max_nc = std::max(b->max_nc, nc * nr);
        st0[i] = c->step;
        hd0[i] = c->head;
        nsl[i] = K;
        const int64_t *dstep = b->steps.as<int64_t>() + i, *dhead = b->heads.as<int64_t>() + i;
        // history group
        const int64_t rt_f = qhp::grouped_rows_per_tile(qhp::GK_F64, nr);
        int64_t ns_max = 1;  // partial sums for the largest split count of any tile shape
        for (int v = 0; v < nvar; ++v)
            ns_max = std::max<int64_t>(ns_max, group_splits(qhp::grouped_rows_per_tile(b->kind, nr, trans, v), ne, K));
        b->part_h[i].alloc(asz * ns_max * ne * nr);
        qhp::GDesc g{};
        g.A = c->slabs.p; g.rows = ne; g.cols = ne; g.ld = ld; g.lag_stride = ne * ld; g.nlags = K;
        g.scales = nullptr;
        g.x = c->ring32.p ? c->ring32.p : c->ring64.p;
        g.x_slot_stride = ld * nr; g.n_slots = K; g.head = dhead; g.x_ld = 0;
        const bool t64 = trans && b->kind == qhp::GK_F32A;
        // ring kept transposed as well (FP32 or, for FP64 y, FP64).  A context
        // that marches FP32 blocks with FP64 y on several right-hand sides
        // keeps such a ring itself: the batch then reads and writes that one, so
        // the context's own steps after the batch see the history the batch made.
        double *ring_t64 = nullptr;
        if (trans) {
            if (t64 && c->ring64t.p) {
                ring_t64 = c->ring64t.as<double>();
                g.x = c->ring64t.p;
            } else {  // a private copy, from the current state
                b->ringt[i].alloc((t64 ? sizeof(double) : sizeof(float)) * K * nr * ld);
                if (t64) qhp::launch_ring_transpose(s, K, ld, nr, c->ring64.as<double>(), b->ringt[i].as<double>());
                else qhp::launch_ring_transpose(s, K, ld, nr, c->ring32.as<float>(), b->ringt[i].as<float>());
                if (t64) ring_t64 = b->ringt[i].as<double>();
                g.x = b->ringt[i].p;
            }
            g.x_ld = ld;
        }
        g.partial = b->part_h[i].p;
        hist_base[q] = g;  // rowblocks, nsplit and tile0 per tile shape below
        b->bvec[i].alloc(sizeof(double) * ne * nr);
        // solve group: y = T_0^{-1} b (FP64, padded copy of the inverse)
        b->tinv[i].alloc(sizeof(double) * ne * ld);
        zero(b->tinv[i], s);
        hip_check(hipMemcpy2DAsync(b->tinv[i].p, sizeof(double) * ld, c->Tinv.p, sizeof(double) * ne,
                                   sizeof(double) * ne, ne, hipMemcpyDeviceToDevice, s), "copy");
        b->part_s[i].alloc(sizeof(double) * ne * nr);
        qhp::GDesc gsv{};
        gsv.A = b->tinv[i].p; gsv.rows = ne; gsv.cols = ne; gsv.ld = ld; gsv.lag_stride = 0; gsv.nlags = 1;
        gsv.x = b->bvec[i].p; gsv.x_slot_stride = 0; gsv.n_slots = 1; gsv.head = nullptr;
        gsv.partial = b->part_s[i].p; gsv.nsplit = 1; gsv.rowblocks = (ne + rt_f - 1) / rt_f; gsv.tile0 = t_s;
        t_s += gsv.rowblocks;
        ds[q] = gsv;
        b->yvec[i].alloc(sizeof(double) * ne * nr);
        fs[i] = qhp::GFin{b->part_s[i].p, 1, ne * nr, nullptr, dstep, b->yvec[i].as<double>()};
        gs[i] = qhp::GStore{b->yvec[i].as<double>(), c->ring64.as<double>(), c->ring32.as<float>(), ld * nr, K,
                            ne * nr, dhead, b->errflag.as<int>(), (trans && !t64) ? b->ringt[i].as<float>() : nullptr,
                            ld, nr, ring_t64};
        // post-processing product z = L_Sigma^+ s (padded copy)
        const int64_t ldc = (nc + 7) / 8 * 8;
        b->lsp[i].alloc(sizeof(double) * nc * ldc);
        zero(b->lsp[i], s);
        hip_check(hipMemcpy2DAsync(b->lsp[i].p, sizeof(double) * ldc, c->LSp.p, sizeof(double) * nc,
                                   sizeof(double) * nc, nc, hipMemcpyDeviceToDevice, s), "copy");
        b->sv[i].alloc(sizeof(double) * nc * nr);
        b->part_p[i].alloc(sizeof(double) * nc * nr);
        b->zc[i].alloc(sizeof(double) * nc * nr);
        qhp::GDesc gp{};
        gp.A = b->lsp[i].p; gp.rows = nc; gp.cols = nc; gp.ld = ldc; gp.lag_stride = 0; gp.nlags = 1;
        gp.x = b->sv[i].p; gp.x_slot_stride = 0; gp.n_slots = 1; gp.head = nullptr;
        gp.partial = b->part_p[i].p; gp.nsplit = 1; gp.rowblocks = (nc + rt_f - 1) / rt_f; gp.tile0 = t_p;
        t_p += gp.rowblocks;
        dp[q] = gp;
        fp[i] = qhp::GFin{b->part_p[i].p, 1, nc * nr, nullptr, dstep, b->zc[i].as<double>()};
        qhp::GPost pp{};
        pp.ne = ne; pp.nc = nc; pp.nrhs = nr; pp.dtn = c->dtn;
        pp.tri_edge = c->args.tri_edge; pp.tri_sign = c->args.tri_sign; pp.cells = c->args.cells;
        pp.ring64 = c->ring64.as<double>(); pp.slot_stride = ld * nr; pp.n_slots = K;
        pp.head = dhead; pp.step = dstep; pp.sv = b->sv[i].as<double>(); pp.z = b->zc[i].as<double>();
        pp.jhist = nullptr;
        b->post_host[i] = pp;
    }
    // history descriptors of one tile shape (rows per tile, splits, tile offsets)
    auto hist_tables = [&](int v) {
        int64_t t = 0;
        for (int q = 0; q < n; ++q) {
            const int i = order[q];
            const qhp_ctx *c = b->ctxs[i];
            const int64_t ne = c->mesh.ne, rt = qhp::grouped_rows_per_tile(b->kind, nr, trans, v);
            qhp::GDesc g = hist_base[q];
            g.nsplit = group_splits(rt, ne, c->K);
            g.rowblocks = (ne + rt - 1) / rt;
            g.tile0 = t;
            t += g.rowblocks * g.nsplit;
            dh[q] = g;
            fh[i] = qhp::GFin{b->part_h[i].p, g.nsplit, ne * nr, c->rhs.as<double>(), b->steps.as<int64_t>() + i,
                              b->bvec[i].as<double>()};
        }
        return t;
    };
    b->counter.alloc(sizeof(unsigned long long));
    // march state first: the autotuning launches read the ring heads
    hip_check(hipMemcpyAsync(b->steps.p, st0.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s), "state");
    hip_check(hipMemcpyAsync(b->heads.p, hd0.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s), "state");
    b->hv = variant >= 0 ? variant : 0;
    if (nvar > 1 && variant < 0) {  // autotune the history tile shape on the batch's own blocks
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
        float best = 1e30f;
        for (int v = 0; v < nvar; ++v) {
            const int64_t tiles = hist_tables(v);
            if (tiles >= ((int64_t)1 << 24)) continue;  // beyond one work-group per tile
            upload(b->d_hist, dh, s);
            auto run = [&]() {
                qhp::launch_grouped_gemv(s, b->kind, nr, b->d_hist.as<qhp::GDesc>(), n, tiles,
                                         b->counter.as<unsigned long long>(), trans, v);
            };
            run();
            hip_check(hipEventRecord(e0, s), "event");
            run();
            run();
            hip_check(hipEventRecord(e1, s), "event");
            hip_check(hipEventSynchronize(e1), "event");
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
            if (c0->verbose)
                std::fprintf(stderr, "[qhp] batch history, %lld rows per tile (%s): %.3f ms\n",
                             (long long)qhp::grouped_rows_per_tile(b->kind, nr, trans, v),
                             qhp::grouped_variant_name(b->kind, nr, trans, v), ms / 2);
            if (ms < best) {
                best = ms;
                b->hv = v;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    t_h = hist_tables(b->hv);
    // the LDS-staged history kernels launch one 256-lane work-group per tile
    if (t_h >= ((int64_t)1 << 24)) throw Fail{QHP_EINVAL, "batch history has too many work tiles"};
    b->tiles_h = t_h;
    b->tiles_s = t_s;
    b->tiles_p = t_p;
    upload(b->d_hist, dh, s);
    upload(b->d_solve, ds, s);
    upload(b->d_post, dp, s);
    upload(b->f_hist, fh, s);
    upload(b->f_solve, fs, s);
    upload(b->f_post, fp, s);
    upload(b->st, gs, s);
    upload(b->po, b->post_host, s);
    upload(b->nslots, nsl, s);
    b->synced.assign(st0.begin(), st0.end());
    hip_check(hipStreamSynchronize(s), "batch set-up");
}

static void enqueue_batch_step(qhp_batch *b)
{
    hipStream_t s = b->s;
    const int n = b->n, nr = b->nrhs;
    qhp::launch_grouped_gemv(s, b->kind, nr, b->d_hist.as<qhp::GDesc>(), n, b->tiles_h, b->counter.as<unsigned long long>(),
                             qhp::grouped_ring_transposed(b->kind, nr), b->hv);
    qhp::launch_grouped_finish(s, b->acc_double, b->f_hist.as<qhp::GFin>(), n, b->max_ne, 0);
    qhp::launch_grouped_gemv(s, qhp::GK_F64, nr, b->d_solve.as<qhp::GDesc>(), n, b->tiles_s, b->counter.as<unsigned long long>(),
                             false);
    qhp::launch_grouped_finish(s, true, b->f_solve.as<qhp::GFin>(), n, b->max_ne, 1);
    qhp::launch_grouped_store(s, b->st.as<qhp::GStore>(), n, b->max_ne);
    qhp::launch_grouped_post(s, 0, b->po.as<qhp::GPost>(), n, b->max_nc);
    qhp::launch_grouped_gemv(s, qhp::GK_F64, nr, b->d_post.as<qhp::GDesc>(), n, b->tiles_p, b->counter.as<unsigned long long>(),
                             false);
    qhp::launch_grouped_finish(s, true, b->f_post.as<qhp::GFin>(), n, b->max_nc, 1);
    qhp::launch_grouped_post(s, 1, b->po.as<qhp::GPost>(), n, b->max_ne);
    qhp::launch_grouped_advance(s, b->steps.as<int64_t>(), b->heads.as<int64_t>(), b->nslots.as<int64_t>(), n);
}

static int batch_kind(int32_t precision)
{
    return precision == QHP_F64 ? qhp::GK_F64 : (precision == QHP_F32 ? qhp::GK_F32 : qhp::GK_F32A);
}

extern "C" int qhp_batch_variants(int32_t precision, int32_t n_rhs)
{
    if (precision != QHP_F64 && precision != QHP_F32 && precision != QHP_F32A) return 0;
    if (n_rhs != 1 && n_rhs != 2 && n_rhs != 4 && n_rhs != 8) return 0;
    const int kind = batch_kind(precision);
    return qhp::grouped_hist_variants(kind, n_rhs, qhp::grouped_ring_transposed(kind, n_rhs));
}

extern "C" int qhp_batch_history_variant(const qhp_batch *b) { return b ? b->hv : -1; }

extern "C" int qhp_batch_create(qhp_ctx *const *ctxs, int32_t n, qhp_batch **out)
{
    return qhp_batch_create_variant(ctxs, n, -1, out);
}

extern "C" int qhp_batch_create_variant(qhp_ctx *const *ctxs, int32_t n, int32_t variant, qhp_batch **out)
{
    QHP_ALLOC_SCOPE((ctxs && n > 0) ? ctxs[0] : nullptr);
    if (!ctxs || n < 1 || !out) return QHP_EINVAL;
    qhp_ctx *c0 = ctxs[0];
    for (int i = 0; i < n; ++i) {
        qhp_ctx *c = ctxs[i];
        if (!c || c->state != 3 || c->broken) return guard(c0, QHP_ESTATE, "every context needs set_incident");
        if (c->p.device != c0->p.device || c->p.precision != c0->p.precision || c->nrhs != c0->nrhs)
            return guard(c0, QHP_EINVAL, "batch contexts must share device, precision and n_rhs");
    }
    if (c0->p.precision == QHP_BF16 || c0->p.precision == QHP_BF16X2 || c0->p.precision == QHP_I8X4 ||
        is_fac(c0->p.precision))
        return guard(c0, QHP_EINVAL, "the batch kernels take F64, F32 or F32A blocks");
    if (c0->nrhs != 1 && c0->nrhs != 2 && c0->nrhs != 4 && c0->nrhs != 8)
        return guard(c0, QHP_EINVAL, "batch n_rhs must be 1, 2, 4 or 8");
    if (variant < -1 || variant >= qhp_batch_variants(c0->p.precision, c0->nrhs))
        return guard(c0, QHP_EINVAL, "no such history tile shape for this precision and n_rhs");
    qhp_batch *b = new qhp_batch();
    try {
        hip_check(hipSetDevice(c0->p.device), "hipSetDevice");
        b->ctxs.assign(ctxs, ctxs + n);
        b->n = n;
        b->nrhs = c0->nrhs;
        b->kind = batch_kind(c0->p.precision);
        b->acc_double = b->kind != qhp::GK_F32;
        hip_check(hipStreamCreateWithFlags(&b->s, hipStreamNonBlocking), "stream");
        for (int i = 0; i < n; ++i) hip_check(hipStreamSynchronize(ctxs[i]->s), "sync");
        build_batch(b, variant);
        // capture one step; every per-step quantity is read from device state
        hip_check(hipStreamBeginCapture(b->s, hipStreamCaptureModeThreadLocal), "capture");
        enqueue_batch_step(b);
        hip_check(hipStreamEndCapture(b->s, &b->graph), "capture");
        hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "instantiate");
    } catch (const Fail &f) {
        delete b;
        return guard(c0, f.code, f.msg);
    }
    for (qhp_ctx *c : b->ctxs) c->batch_refs += 1;
    b->held = b->ctxs;
    *out = b;
    return QHP_OK;
}

extern "C" int qhp_batch_run(qhp_batch *b, int32_t n_steps, double *const *j_hists)
{
    QHP_ALLOC_SCOPE((b && !b->ctxs.empty()) ? b->ctxs[0] : nullptr);
    if (!b || n_steps < 0) return QHP_EINVAL;
    for (qhp_ctx *c : b->ctxs)
        if (c->step + n_steps > c->n_steps) return bguard(b, QHP_EINVAL, "past the last right-hand side");
    try {
        hipStream_t s = b->s;
        // contexts that marched on their own since the batch last ran: bring
        // the device step and ring head, and any private transposed ring, up to date
        for (int i = 0; i < b->n; ++i) {
            qhp_ctx *c = b->ctxs[i];
            if (c->step == b->synced[i]) continue;
            hip_check(hipStreamSynchronize(c->s), "sync");
            const int64_t st = c->step, hd = c->head;
            hip_check(hipMemcpyAsync(b->steps.as<int64_t>() + i, &st, sizeof(int64_t), hipMemcpyHostToDevice, s), "state");
            hip_check(hipMemcpyAsync(b->heads.as<int64_t>() + i, &hd, sizeof(int64_t), hipMemcpyHostToDevice, s), "state");
            if (b->ringt[i].p) {
                if (b->kind == qhp::GK_F32A)
                    qhp::launch_ring_transpose(s, c->K, c->ld, b->nrhs, c->ring64.as<double>(), b->ringt[i].as<double>());
                else
                    qhp::launch_ring_transpose(s, c->K, c->ld, b->nrhs, c->ring32.as<float>(), b->ringt[i].as<float>());
            }
            hip_check(hipStreamSynchronize(s), "state");
            b->synced[i] = st;
        }
        // per-run output pointers: step s of the context writes j_hists[i] + (s - step0) * ne * nrhs
        for (int i = 0; i < b->n; ++i) {
            qhp_ctx *c = b->ctxs[i];
            const int64_t stride = c->mesh.ne * b->nrhs;
            b->post_host[i].jhist = (j_hists && j_hists[i]) ? j_hists[i] - c->step * stride : nullptr;
        }
        hip_check(hipMemcpyAsync(b->po.p, b->post_host.data(), sizeof(qhp::GPost) * b->n, hipMemcpyHostToDevice, s), "post");
        std::vector<hipEvent_t> ev(n_steps + 1);
        for (auto &e : ev) hip_check(hipEventCreate(&e), "event");
        hip_check(hipEventRecord(ev[0], s), "event");
        for (int t = 0; t < n_steps; ++t) {
            hip_check(hipGraphLaunch(b->exec, s), "graph launch");
            hip_check(hipEventRecord(ev[t + 1], s), "event");
        }
        hip_check(hipStreamSynchronize(s), "batch march");
        b->step_ms.resize(n_steps);
        for (int t = 0; t < n_steps; ++t) hip_check(hipEventElapsedTime(&b->step_ms[t], ev[t], ev[t + 1]), "event");
        for (auto e : ev) (void)hipEventDestroy(e);
        std::vector<int64_t> heads(b->n);
        hip_check(hipMemcpy(heads.data(), b->heads.p, sizeof(int64_t) * b->n, hipMemcpyDeviceToHost), "state");
        int e = 0;
        hip_check(hipMemcpy(&e, b->errflag.p, sizeof(int), hipMemcpyDeviceToHost), "flag");
        for (int i = 0; i < b->n; ++i) {
            b->ctxs[i]->step += n_steps;
            b->ctxs[i]->head = heads[i];
            b->synced[i] = b->ctxs[i]->step;
        }
        if (e) return bguard(b, QHP_EUNSTABLE, "non-finite value in a batch member");
    } catch (const Fail &f) {
        return bguard(b, f.code, f.msg);
    }
    return QHP_OK;
}

extern "C" int qhp_batch_step_times(const qhp_batch *b, float *ms, int32_t n)
{
    if (!b || !ms) return QHP_EINVAL;
    for (int i = 0; i < n && i < (int)b->step_ms.size(); ++i) ms[i] = b->step_ms[i];
    return QHP_OK;
}

extern "C" const char *qhp_batch_last_error(const qhp_batch *b) { return b ? b->err.c_str() : "null batch"; }

extern "C" void qhp_batch_destroy(qhp_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->s);
    delete b;
}
