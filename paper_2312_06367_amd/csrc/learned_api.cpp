// C ABI of the learned warm start and of the iterative T_0 solve it feeds:
// loop/star/harmonic coordinates of a context's mesh, the perceptron (its
// parameters, forward and backward passes, Adam, training on march
// histories) and restarted GMRES with FP64 residual refinement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "ctx.h"
#include "learned.h"
#include "linalg.h"
#include "march.h"

using qhp::DBuf;
using qhp::Fail;
using qhp::hip_check;
using qhp::upload;
using qhp::zero;

struct qhp_mlp {
    qhp_ctx *ctx = nullptr;
    hipStream_t s = nullptr;
    int64_t nf = 0, nin = 0, hid = 0, nparam = 0;
    int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
    DBuf P, Pb, G, Mo, Vo;  // FP32 master parameters, BF16 copy, gradient, Adam moments
    int64_t adam_t = 0;
    int64_t cap = 0;  // batch capacity of the work buffers
    DBuf X, T, Z1, A1, A1b, Z2, A2, A2b, O, dO, dA, dZ, loss, sig, fg;
    std::string err;
    const uint16_t *W(int64_t off) const { return Pb.as<uint16_t>() + off; }
    const float *Pf(int64_t off) const { return P.as<float>() + off; }
    float *Gf(int64_t off) const { return G.as<float>() + off; }
};

static int mguard(qhp_mlp *m, int code, const std::string &msg)
{
    if (m) m->err = msg;
    return code;
}

// ------------------------------------------------------------------ loop/star
namespace qhp {

// Orthonormal basis of the harmonic space range(I - P^Sigma - P^Lambda):
// the projector applied to N_H + 4 random vectors, then modified
// Gram-Schmidt (two passes) on the host, keeping the N_H directions found.
static void harmonic_basis(qhp_ctx *c)
{
    const int64_t ne = c->mesh.ne, nh = c->mesh.n_harmonic;
    c->ls_nh = nh;
    if (nh == 0) return;
    if (!c->PS.p || !c->PPL.p) throw Fail{QHP_ESTATE, "projectors were released"};
    const int64_t p = nh + 4;
    std::mt19937_64 gen(0x5eed);
    std::normal_distribution<double> nd;
    std::vector<double> R((size_t)ne * p);
    for (auto &v : R) v = nd(gen);
    DBuf dR, t1, t2;
    upload(dR, R, c->s);
    t1.alloc(sizeof(double) * ne * p);
    t2.alloc(sizeof(double) * ne * p);
    gemm_f64(c->s, false, false, ne, p, ne, 1.0, c->PS.as<double>(), ne, dR.as<double>(), p, 0.0, t1.as<double>(), p);
    gemm_f64(c->s, false, false, ne, p, ne, 1.0, c->PPL.as<double>(), ne, dR.as<double>(), p, 0.0, t2.as<double>(), p);
    axpby(c->s, ne * p, 1.0, dR.as<double>(), -1.0, t1.as<double>(), dR.as<double>());
    axpby(c->s, ne * p, 1.0, dR.as<double>(), -1.0, t2.as<double>(), dR.as<double>());
    hip_check(hipMemcpyAsync(R.data(), dR.p, sizeof(double) * ne * p, hipMemcpyDeviceToHost, c->s), "harmonic");
    hip_check(hipStreamSynchronize(c->s), "harmonic");
    std::vector<double> H((size_t)ne * nh, 0.0);
    std::vector<std::vector<double>> basis;
    for (int64_t j = 0; j < p && (int64_t)basis.size() < nh; ++j) {
        std::vector<double> v(ne);
        for (int64_t i = 0; i < ne; ++i) v[i] = R[i * p + j];
        double n0 = std::sqrt(std::inner_product(v.begin(), v.end(), v.begin(), 0.0));
        for (int pass = 0; pass < 2; ++pass)
            for (auto &b : basis) {
                double d = std::inner_product(v.begin(), v.end(), b.begin(), 0.0);
                for (int64_t i = 0; i < ne; ++i) v[i] -= d * b[i];
            }
        double n1 = std::sqrt(std::inner_product(v.begin(), v.end(), v.begin(), 0.0));
        if (!(n1 > 1e-6 * n0)) continue;
        for (auto &x : v) x /= n1;
        basis.push_back(std::move(v));
    }
    if ((int64_t)basis.size() != nh) throw Fail{QHP_EMESH, "harmonic space smaller than the genus implies"};
    for (int64_t j = 0; j < nh; ++j)
        for (int64_t i = 0; i < ne; ++i) H[i * nh + j] = basis[j][i];
    upload(c->Hb, H, c->s);
    hip_check(hipStreamSynchronize(c->s), "harmonic");
}

void loopstar_prepare(qhp_ctx *c)
{
    if (c->ls_nh >= 0) return;
    if (!c->LSp.p || !c->LLp.p) throw Fail{QHP_ESTATE, "assemble first"};
    harmonic_basis(c);
}

// F [n][ldf] = [l | s | h] of Y [n][ldy]
void loopstar_features(qhp_ctx *c, const double *Y, int64_t n, int64_t ldy, double *F, int64_t ldf)
{
    loopstar_prepare(c);
    const qhp::Mesh &m = c->mesh;
    const int64_t ne = m.ne, nc = m.nc, nv = m.nv, nh = c->ls_nh;
    if (c->ls_cap < n) {
        c->ls_sig.alloc(sizeof(double) * n * nc);
        c->ls_lam.alloc(sizeof(double) * n * nv);
        c->ls_cap = n;
    }
    const AsmArgs &a = c->args;
    launch_incidence_t(c->s, n, ne, nc, nv, a.tri_edge, a.tri_sign, a.vedge_off, a.vedge, a.edges, Y, ldy,
                       c->ls_sig.as<double>(), c->ls_lam.as<double>());
    if (n == 1) {
        launch_gemv_f64(c->s, nv, c->LLp.as<double>(), c->ls_lam.as<double>(), F);
        launch_gemv_f64(c->s, nc, c->LSp.as<double>(), c->ls_sig.as<double>(), F + nv);
    } else {  // both pseudo-inverses are symmetric
        gemm_f64(c->s, false, false, n, nv, nv, 1.0, c->ls_lam.as<double>(), nv, c->LLp.as<double>(), nv, 0.0, F, ldf);
        gemm_f64(c->s, false, false, n, nc, nc, 1.0, c->ls_sig.as<double>(), nc, c->LSp.as<double>(), nc, 0.0, F + nv,
                 ldf);
    }
    if (nh > 0)
        gemm_f64(c->s, false, false, n, nh, ne, 1.0, Y, ldy, c->Hb.as<double>(), nh, 0.0, F + nv + nc, ldf);
}

void loopstar_reconstruct(qhp_ctx *c, const double *F, int64_t n, int64_t ldf, double *Y, int64_t ldy)
{
    loopstar_prepare(c);
    const qhp::Mesh &m = c->mesh;
    launch_reconstruct(c->s, n, m.ne, m.nv, m.nc, c->ls_nh, c->args.edges, c->args.cells, c->Hb.as<double>(), F, ldf,
                       Y, ldy);
}

}  // namespace qhp

// ------------------------------------------------------------------ perceptron
static void mlp_reserve(qhp_mlp *m, int64_t B)
{
    if (B <= m->cap) return;
    const int64_t nf = m->nf, nin = m->nin, hid = m->hid;
    m->X.alloc(sizeof(uint16_t) * B * nin);
    m->T.alloc(sizeof(float) * B * nf);
    m->Z1.alloc(sizeof(float) * B * hid);
    m->A1.alloc(sizeof(float) * B * hid);
    m->A1b.alloc(sizeof(uint16_t) * B * hid);
    m->Z2.alloc(sizeof(float) * B * hid);
    m->A2.alloc(sizeof(float) * B * hid);
    m->A2b.alloc(sizeof(uint16_t) * B * hid);
    m->O.alloc(sizeof(float) * B * nf);
    m->dO.alloc(sizeof(float) * B * nf);
    m->dA.alloc(sizeof(float) * B * hid);
    m->dZ.alloc(sizeof(float) * B * hid);
    m->cap = B;
}

// C = op product with a K split chosen to give the chip about a thousand
// work-groups; a split product accumulates atomically into a zeroed C
static void gemm(hipStream_t s, int64_t M, int64_t N, int64_t K, int ta, const void *A, int64_t sam, int64_t sak,
                 int tb, const void *B, int64_t sbk, int64_t sbn, float *C, int64_t ldc)
{
    const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64);
    int64_t ks = std::max<int64_t>(1, std::min<int64_t>(1024 / std::max<int64_t>(tiles, 1), K / 256));
    if (ks > 1) {
        if (ldc == N) qhp::launch_fill_f32(s, M * N, 0.f, C);
        else
            for (int64_t i = 0; i < M; ++i) qhp::launch_fill_f32(s, N, 0.f, C + i * ldc);
    }
    qhp::mlp_gemm(s, M, N, K, 1.f, ta, A, sam, sak, tb, B, sbk, sbn, 0.f, C, ldc, (int)ks);
}

static void mlp_forward(qhp_mlp *m, int64_t B, int tx, const void *X)
{
    hipStream_t s = m->s;
    const int64_t nf = m->nf, nin = m->nin, hid = m->hid;
    using qhp::MT_BF16;
    gemm(s, B, hid, nin, tx, X, nin, 1, MT_BF16, m->W(m->oW1), 1, nin, m->Z1.as<float>(), hid);
    qhp::launch_bias_tanh(s, B, hid, m->Z1.as<float>(), m->Pf(m->ob1), m->A1.as<float>(), m->A1b.as<uint16_t>());
    gemm(s, B, hid, hid, MT_BF16, m->A1b.p, hid, 1, MT_BF16, m->W(m->oW2), 1, hid, m->Z2.as<float>(), hid);
    qhp::launch_bias_tanh(s, B, hid, m->Z2.as<float>(), m->Pf(m->ob2), m->A2.as<float>(), m->A2b.as<uint16_t>());
    gemm(s, B, nf, hid, MT_BF16, m->A2b.p, hid, 1, MT_BF16, m->W(m->oW3), 1, hid, m->O.as<float>(), nf);
    qhp::launch_bias_add(s, B, nf, m->O.as<float>(), m->Pf(m->ob3));
}

// gradient of the mean squared error of the last forward pass against T;
// the batch loss is added to *loss (device)
static void mlp_backward(qhp_mlp *m, int64_t B, int tx, const void *X, const float *T)
{
    hipStream_t s = m->s;
    const int64_t nf = m->nf, nin = m->nin, hid = m->hid;
    using qhp::MT_BF16;
    using qhp::MT_F32;
    qhp::launch_mse_grad(s, B * nf, m->O.as<float>(), T, m->dO.as<float>(), m->loss.as<double>());
    gemm(s, nf, hid, B, MT_F32, m->dO.p, 1, nf, MT_F32, m->A2.p, hid, 1, m->Gf(m->oW3), hid);
    qhp::launch_col_sum(s, B, nf, m->dO.as<float>(), m->Gf(m->ob3));
    gemm(s, B, hid, nf, MT_F32, m->dO.p, nf, 1, MT_BF16, m->W(m->oW3), hid, 1, m->dA.as<float>(), hid);
    qhp::launch_tanh_back(s, B * hid, m->dA.as<float>(), m->A2.as<float>(), m->dZ.as<float>());
    gemm(s, hid, hid, B, MT_F32, m->dZ.p, 1, hid, MT_F32, m->A1.p, hid, 1, m->Gf(m->oW2), hid);
    qhp::launch_col_sum(s, B, hid, m->dZ.as<float>(), m->Gf(m->ob2));
    gemm(s, B, hid, hid, MT_F32, m->dZ.p, hid, 1, MT_BF16, m->W(m->oW2), hid, 1, m->dA.as<float>(), hid);
    qhp::launch_tanh_back(s, B * hid, m->dA.as<float>(), m->A1.as<float>(), m->dZ.as<float>());
    gemm(s, hid, nin, B, MT_F32, m->dZ.p, 1, hid, tx, X, nin, 1, m->Gf(m->oW1), nin);
    qhp::launch_col_sum(s, B, hid, m->dZ.as<float>(), m->Gf(m->ob1));
}

static void mlp_adam(qhp_mlp *m, double lr, double b1, double b2, double eps)
{
    m->adam_t += 1;
    const double t = (double)m->adam_t;
    const double c2 = std::sqrt(1.0 - std::pow(b2, t));
    const double lr_t = lr * c2 / (1.0 - std::pow(b1, t));
    qhp::launch_adam(m->s, m->nparam, m->P.as<float>(), m->G.as<float>(), m->Mo.as<float>(), m->Vo.as<float>(),
                     (float)lr_t, (float)b1, (float)b2, (float)(eps * c2), m->Pb.as<uint16_t>());
}

// guess of f_i from f1 = f_{i-1} .. f4 = f_{i-4} (device FP64) into g
static void mlp_guess(qhp_mlp *m, const double *f1, const double *f2, const double *f3, const double *f4, double *g)
{
    hipStream_t s = m->s;
    qhp::launch_window_x(s, m->nf, f1, f2, f3, f4, m->X.as<uint16_t>(), m->sig.as<double>());
    mlp_forward(m, 1, qhp::MT_BF16, m->X.p);
    qhp::launch_guess(s, m->nf, f1, f2, f3, m->sig.as<double>(), m->O.as<float>(), g);
}

extern "C" int qhp_mlp_create(qhp_ctx *ctx, int32_t hidden, uint64_t seed, qhp_mlp **out)
{
    QHP_ALLOC_SCOPE(ctx);
    if (!ctx || !out || hidden < 1) return QHP_EINVAL;
    if (ctx->state < 2) return guard(ctx, QHP_ESTATE, "assemble first");
    qhp_mlp *m = new qhp_mlp();
    try {
        hip_check(hipSetDevice(ctx->p.device), "hipSetDevice");
        qhp::loopstar_prepare(ctx);
        m->ctx = ctx;
        m->s = ctx->s;
        m->nf = ctx->mesh.nv + ctx->mesh.nc + ctx->ls_nh;
        m->nin = 4 * m->nf;
        m->hid = hidden;
        const int64_t nf = m->nf, nin = m->nin, hid = m->hid;
        m->oW1 = 0;
        m->ob1 = m->oW1 + hid * nin;
        m->oW2 = m->ob1 + hid;
        m->ob2 = m->oW2 + hid * hid;
        m->oW3 = m->ob2 + hid;
        m->ob3 = m->oW3 + nf * hid;
        m->nparam = m->ob3 + nf;
        m->P.alloc(sizeof(float) * m->nparam);
        m->Pb.alloc(sizeof(uint16_t) * m->nparam);
        m->G.alloc(sizeof(float) * m->nparam);
        m->Mo.alloc(sizeof(float) * m->nparam);
        m->Vo.alloc(sizeof(float) * m->nparam);
        m->loss.alloc(sizeof(double));
        m->sig.alloc(sizeof(double));
        m->fg.alloc(sizeof(double) * nf);
        hipStream_t s = m->s;
        // Glorot-uniform weights, zero biases; the output layer starts small so
        // the untrained network is close to linear extrapolation
        qhp::launch_fill_f32(s, m->nparam, 0.f, m->P.as<float>());
        qhp::launch_init_uniform(s, hid * nin, (float)std::sqrt(6.0 / (nin + hid)), seed, 0, m->P.as<float>() + m->oW1);
        qhp::launch_init_uniform(s, hid * hid, (float)std::sqrt(6.0 / (2 * hid)), seed, (uint64_t)m->oW2,
                                 m->P.as<float>() + m->oW2);
        qhp::launch_init_uniform(s, nf * hid, (float)(0.01 * std::sqrt(6.0 / (hid + nf))), seed, (uint64_t)m->oW3,
                                 m->P.as<float>() + m->oW3);
        qhp::launch_to_bf16(s, m->nparam, m->P.as<float>(), m->Pb.as<uint16_t>());
        qhp::launch_fill_f32(s, m->nparam, 0.f, m->Mo.as<float>());
        qhp::launch_fill_f32(s, m->nparam, 0.f, m->Vo.as<float>());
        mlp_reserve(m, 1);
        hip_check(hipStreamSynchronize(s), "perceptron set-up");
    } catch (const Fail &f) {
        delete m;
        return guard(ctx, f.code, f.msg);
    }
    *out = m;
    return QHP_OK;
}

extern "C" void qhp_mlp_destroy(qhp_mlp *m)
{
    if (!m) return;
    if (m->ctx && m->ctx->mlp == m) m->ctx->mlp = nullptr;
    (void)hipStreamSynchronize(m->s);
    delete m;
}

extern "C" const char *qhp_mlp_last_error(const qhp_mlp *m) { return m ? m->err.c_str() : "null perceptron"; }

extern "C" int qhp_mlp_dims(const qhp_mlp *m, int64_t *n_features, int64_t *n_params, int64_t *hidden)
{
    if (!m) return QHP_EINVAL;
    if (n_features) *n_features = m->nf;
    if (n_params) *n_params = m->nparam;
    if (hidden) *hidden = m->hid;
    return QHP_OK;
}

extern "C" int qhp_mlp_set_params(qhp_mlp *m, const float *params)
{
    QHP_ALLOC_SCOPE(m ? m->ctx : nullptr);
    if (!m || !params) return QHP_EINVAL;
    try {
        hip_check(hipMemcpyAsync(m->P.p, params, sizeof(float) * m->nparam, hipMemcpyHostToDevice, m->s), "params");
        qhp::launch_to_bf16(m->s, m->nparam, m->P.as<float>(), m->Pb.as<uint16_t>());
        qhp::launch_fill_f32(m->s, m->nparam, 0.f, m->Mo.as<float>());
        qhp::launch_fill_f32(m->s, m->nparam, 0.f, m->Vo.as<float>());
        m->adam_t = 0;
        hip_check(hipStreamSynchronize(m->s), "params");
    } catch (const Fail &f) {
        return mguard(m, f.code, f.msg);
    }
    return QHP_OK;
}

extern "C" int qhp_mlp_get_params(const qhp_mlp *m, float *params)
{
    if (!m || !params) return QHP_EINVAL;
    if (hipStreamSynchronize(m->s) != hipSuccess ||
        hipMemcpy(params, m->P.p, sizeof(float) * m->nparam, hipMemcpyDeviceToHost) != hipSuccess)
        return QHP_EDEVICE;
    return QHP_OK;
}

extern "C" int qhp_mlp_forward(qhp_mlp *m, const float *x, int32_t batch, float *out)
{
    QHP_ALLOC_SCOPE(m ? m->ctx : nullptr);
    if (!m || !x || !out || batch < 1) return QHP_EINVAL;
    try {
        mlp_reserve(m, batch);
        mlp_forward(m, batch, qhp::MT_F32, x);
        hip_check(hipMemcpyAsync(out, m->O.p, sizeof(float) * batch * m->nf, hipMemcpyDeviceToDevice, m->s), "out");
        hip_check(hipStreamSynchronize(m->s), "forward");
    } catch (const Fail &f) {
        return mguard(m, f.code, f.msg);
    }
    return QHP_OK;
}

extern "C" int qhp_mlp_loss_grad(qhp_mlp *m, const float *x, const float *t, int32_t batch, double *loss,
                                 float *grad)
{
    QHP_ALLOC_SCOPE(m ? m->ctx : nullptr);
    if (!m || !x || !t || batch < 1) return QHP_EINVAL;
    try {
        mlp_reserve(m, batch);
        qhp::launch_fill_f64(m->s, 1, 0.0, m->loss.as<double>());
        mlp_forward(m, batch, qhp::MT_F32, x);
        mlp_backward(m, batch, qhp::MT_F32, x, t);
        if (loss) hip_check(hipMemcpyAsync(loss, m->loss.p, sizeof(double), hipMemcpyDeviceToHost, m->s), "loss");
        if (grad)
            hip_check(hipMemcpyAsync(grad, m->G.p, sizeof(float) * m->nparam, hipMemcpyDeviceToHost, m->s), "grad");
        hip_check(hipStreamSynchronize(m->s), "backward");
    } catch (const Fail &f) {
        return mguard(m, f.code, f.msg);
    }
    return QHP_OK;
}

extern "C" int qhp_mlp_adam(qhp_mlp *m, double lr, double beta1, double beta2, double eps)
{
    QHP_ALLOC_SCOPE(m ? m->ctx : nullptr);
    if (!m || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps >= 0.0))
        return QHP_EINVAL;
    mlp_adam(m, lr, beta1, beta2, eps);
    return hipStreamSynchronize(m->s) == hipSuccess ? QHP_OK : QHP_EDEVICE;
}

extern "C" int qhp_mlp_guess(qhp_mlp *m, const double *f, double *g)
{
    QHP_ALLOC_SCOPE(m ? m->ctx : nullptr);
    if (!m || !f || !g) return QHP_EINVAL;
    try {
        const int64_t nf = m->nf;
        mlp_guess(m, f, f + nf, f + 2 * nf, f + 3 * nf, g);
        hip_check(hipStreamSynchronize(m->s), "guess");
    } catch (const Fail &e) {
        return mguard(m, e.code, e.msg);
    }
    return QHP_OK;
}

extern "C" int qhp_mlp_features(qhp_mlp *m, const double *y, int64_t n, double *f)
{
    QHP_ALLOC_SCOPE(m ? m->ctx : nullptr);
    if (!m || !y || !f || n < 1) return QHP_EINVAL;
    try {
        qhp::loopstar_features(m->ctx, y, n, m->ctx->mesh.ne, f, m->nf);
        hip_check(hipStreamSynchronize(m->s), "features");
    } catch (const Fail &e) {
        return mguard(m, e.code, e.msg);
    }
    return QHP_OK;
}

extern "C" int qhp_mlp_reconstruct(qhp_mlp *m, const double *f, int64_t n, double *y)
{
    QHP_ALLOC_SCOPE(m ? m->ctx : nullptr);
    if (!m || !y || !f || n < 1) return QHP_EINVAL;
    try {
        qhp::loopstar_reconstruct(m->ctx, f, n, m->nf, y, m->ctx->mesh.ne);
        hip_check(hipStreamSynchronize(m->s), "reconstruct");
    } catch (const Fail &e) {
        return mguard(m, e.code, e.msg);
    }
    return QHP_OK;
}

extern "C" int qhp_mlp_train(qhp_mlp *m, const double *y, int64_t n_runs, int64_t n_steps, int32_t epochs,
                             int32_t batch, double lr, uint64_t seed, double *epoch_loss)
{
    QHP_ALLOC_SCOPE(m ? m->ctx : nullptr);
    if (!m || !y || n_runs < 1 || n_steps < 6 || epochs < 1 || batch < 1 || !(lr > 0.0)) return QHP_EINVAL;
    try {
        qhp_ctx *c = m->ctx;
        hipStream_t s = m->s;
        const int64_t ne = c->mesh.ne, nf = m->nf;
        // features of every step, rows ordered [step][run]
        DBuf F, Yt, sig;
        F.alloc(sizeof(double) * n_steps * n_runs * nf);
        const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n_steps, ((int64_t)1 << 27) / (ne * n_runs)));
        Yt.alloc(sizeof(double) * chunk * n_runs * ne);
        for (int64_t t0 = 0; t0 < n_steps; t0 += chunk) {
            const int64_t nt = std::min(chunk, n_steps - t0);
            for (int64_t t = 0; t < nt; ++t)  // [ne][n_runs] -> [n_runs][ne]
                qhp::transpose_f64(s, ne, n_runs, y + (t0 + t) * ne * n_runs, n_runs,
                                   Yt.as<double>() + t * n_runs * ne, ne);
            qhp::loopstar_features(c, Yt.as<double>(), nt * n_runs, ne, F.as<double>() + t0 * n_runs * nf, nf);
        }
        sig.alloc(sizeof(double) * n_steps * n_runs);
        qhp::launch_rms_d3(s, n_steps * n_runs, nf, F.as<double>(), n_runs, sig.as<double>());
        std::vector<double> hs(n_steps * n_runs);
        hip_check(hipMemcpyAsync(hs.data(), sig.p, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, s), "rms");
        hip_check(hipStreamSynchronize(s), "rms");
        // sample (run, i): target step i >= 4 (0-based), window rows i-1..i-4,
        // kept when the third difference of the window is not zero
        std::vector<int64_t> samples;
        for (int64_t i = 4; i < n_steps; ++i)
            for (int64_t r = 0; r < n_runs; ++r) {
                const double sg = hs[(i - 1) * n_runs + r];
                if (std::isfinite(sg) && sg > 1e-250) samples.push_back((i - 1) * n_runs + r);
            }
        if (samples.empty()) return mguard(m, QHP_EINVAL, "no usable training windows");
        mlp_reserve(m, batch);
        DBuf idx;
        idx.alloc(sizeof(int64_t) * samples.size());
        std::mt19937_64 gen(seed);
        for (int32_t ep = 0; ep < epochs; ++ep) {
            std::shuffle(samples.begin(), samples.end(), gen);
            hip_check(hipMemcpyAsync(idx.p, samples.data(), sizeof(int64_t) * samples.size(), hipMemcpyHostToDevice, s),
                      "samples");
            qhp::launch_fill_f64(s, 1, 0.0, m->loss.as<double>());
            int64_t nb = 0;
            for (size_t b0 = 0; b0 < samples.size(); b0 += batch) {
                const int64_t B = std::min<int64_t>(batch, (int64_t)(samples.size() - b0));
                qhp::launch_gather_windows(s, B, nf, F.as<double>(), n_runs, idx.as<int64_t>() + b0,
                                           m->X.as<uint16_t>(), m->T.as<float>());
                mlp_forward(m, B, qhp::MT_BF16, m->X.p);
                mlp_backward(m, B, qhp::MT_BF16, m->X.p, m->T.as<float>());
                mlp_adam(m, lr, 0.9, 0.999, 1e-8);
                ++nb;
            }
            double l = 0.0;
            hip_check(hipMemcpyAsync(&l, m->loss.p, sizeof(double), hipMemcpyDeviceToHost, s), "loss");
            hip_check(hipStreamSynchronize(s), "epoch");
            if (epoch_loss) epoch_loss[ep] = l / (double)nb;
        }
    } catch (const Fail &f) {
        return mguard(m, f.code, f.msg);
    }
    return QHP_OK;
}

extern "C" int qhp_attach_mlp(qhp_ctx *ctx, qhp_mlp *m)
{
    QHP_ALLOC_SCOPE(ctx);
    if (!ctx) return QHP_EINVAL;
    if (m && m->ctx != ctx) return guard(ctx, QHP_EINVAL, "the perceptron was built for another context");
    ctx->mlp = m;
    return QHP_OK;
}

// ------------------------------------------------------------------ GMRES
namespace qhp {

void gmres_prepare(qhp_ctx *c)
{
    const int64_t ne = c->mesh.ne, ld = c->ld, m = c->gm_m;
    if (!c->T0raw.p) throw Fail{QHP_ESTATE, "T_0 was released"};
    hipStream_t s = c->s;
    if (!c->T0f.p) {
        c->T0f.alloc(sizeof(float) * ne * ld);
        launch_quantise_slab(s, ne, ld, c->T0raw.as<double>(), ne, nullptr, QHP_F32, 1.0f, c->T0f.p);
    }
    c->gm_V.alloc(sizeof(float) * (m + 1) * ld);
    c->gm_w.alloc(sizeof(float) * ld);
    c->gm_h1.alloc(sizeof(double) * (m + 1));
    c->gm_h2.alloc(sizeof(double) * (m + 1));
    c->gm_nrm.alloc(sizeof(double) * 2);
    c->gm_R.alloc(sizeof(double) * m * (m + 1));
    c->gm_cs.alloc(sizeof(double) * m);
    c->gm_sn.alloc(sizeof(double) * m);
    c->gm_g.alloc(sizeof(double) * (m + 1));
    c->gm_inv.alloc(sizeof(double));
    c->gm_y.alloc(sizeof(double) * m);
    c->gm_r.alloc(sizeof(double) * ne);
    c->gm_x0.alloc(sizeof(double) * ne);
    if (!c->gm_host) {
        void *p = nullptr;
        hip_check(hipHostMalloc(&p, 6 * sizeof(double), hipHostMallocDefault), "pinned scalars");
        c->gm_host = (double *)p;
    }
    if (c->warm == QHP_WARM_MLP || c->warm == QHP_WARM_BEST) {
        if (!c->mlp) throw Fail{QHP_ESTATE, "no perceptron attached"};
        c->feat.alloc(sizeof(double) * 4 * c->mlp->nf);
    }
    hip_check(hipStreamSynchronize(s), "GMRES set-up");
}

// y_{i-1} and y_{i-2} of the single right-hand side, or null
static const double *ring_y(qhp_ctx *c, int back)
{
    if (c->step < back) return nullptr;
    const int64_t slot = (c->head + back - 1) % c->K;
    return c->ring64.as<double>() + slot * c->ld;
}

static void warm_guess(qhp_ctx *c, int mode, const double *y1, const double *y2, const double *y3, double *x0);

void warm_start(qhp_ctx *c, const double *b, double *x0)
{
    hipStream_t s = c->s;
    const int64_t ne = c->mesh.ne;
    const double *y1 = ring_y(c, 1), *y2 = ring_y(c, 2);
    const double *y3 = ring_y(c, 3);
    int mode = c->warm;
    if ((mode == QHP_WARM_MLP || mode == QHP_WARM_BEST) && (!c->mlp || c->feat_n < 4)) mode = QHP_WARM_QUAD;
    if (mode == QHP_WARM_BEST) {  // both guesses, the one with the smaller FP64 residual
        warm_guess(c, QHP_WARM_MLP, y1, y2, y3, x0);
        double *xq = c->gm_x0.as<double>();
        warm_guess(c, QHP_WARM_QUAD, y1, y2, y3, xq);
        launch_gm_residual(s, ne, c->T0raw.as<double>(), x0, b, c->gm_r.as<double>(), c->gm_nrm.as<double>(),
                           c->gm_host + 4);
        launch_gm_residual(s, ne, c->T0raw.as<double>(), xq, b, c->gm_r.as<double>(), c->gm_nrm.as<double>(),
                           c->gm_host + 5);
        hip_check(hipStreamSynchronize(s), "warm start");
        volatile double *hv = c->gm_host;
        if (hv[5] < hv[4])
            hip_check(hipMemcpyAsync(x0, xq, sizeof(double) * ne, hipMemcpyDeviceToDevice, s), "warm start");
        else
            c->gm_net_starts += 1;
        return;
    }
    warm_guess(c, mode, y1, y2, y3, x0);
}

static void warm_guess(qhp_ctx *c, int mode, const double *y1, const double *y2, const double *y3, double *x0)
{
    hipStream_t s = c->s;
    const int64_t ne = c->mesh.ne;
    if (mode == QHP_WARM_QUAD && !y3) mode = QHP_WARM_EXTRAP;
    if (mode == QHP_WARM_EXTRAP && !y2) mode = QHP_WARM_PREV;
    if (mode == QHP_WARM_PREV && !y1) mode = QHP_WARM_COLD;
    switch (mode) {
    case QHP_WARM_COLD: launch_fill_f64(s, ne, 0.0, x0); break;
    case QHP_WARM_PREV:
        hip_check(hipMemcpyAsync(x0, y1, sizeof(double) * ne, hipMemcpyDeviceToDevice, s), "warm start");
        break;
    case QHP_WARM_EXTRAP: axpby(s, ne, 2.0, y1, -1.0, y2, x0); break;
    case QHP_WARM_QUAD:
        axpby(s, ne, 3.0, y1, -3.0, y2, x0);
        axpby(s, ne, 1.0, x0, 1.0, y3, x0);
        break;
    default: {
        qhp_mlp *m = c->mlp;
        const int64_t nf = m->nf, n = c->feat_n;
        const double *F = c->feat.as<double>();
        mlp_guess(m, F + ((n - 1) % 4) * nf, F + ((n - 2) % 4) * nf, F + ((n - 3) % 4) * nf, F + ((n - 4) % 4) * nf,
                  m->fg.as<double>());
        loopstar_reconstruct(c, m->fg.as<double>(), 1, nf, x0, ne);
    }
    }
}

void warm_record(qhp_ctx *c, const double *y)
{
    if ((c->warm != QHP_WARM_MLP && c->warm != QHP_WARM_BEST) || !c->mlp) return;
    const int64_t nf = c->mlp->nf;
    loopstar_features(c, y, 1, c->mesh.ne, c->feat.as<double>() + (c->feat_n % 4) * nf, nf);
    c->feat_n += 1;
}

// x: start on entry, solution on exit.  Returns false if the FP64 residual
// bound was not reached within the refinement budget.
bool gmres_solve(qhp_ctx *c, const double *b, double *x, int32_t *iters, float *res0)
{
    hipStream_t s = c->s;
    const int64_t ne = c->mesh.ne, ld = c->ld;
    const int m = c->gm_m;
    volatile double *hv = c->gm_host;
    launch_norm2(s, ne, b, c->gm_nrm.as<double>() + 1, c->gm_host + 2);
    hip_check(hipStreamSynchronize(s), "GMRES");
    const double nb = std::sqrt(hv[2]);
    *iters = 0;
    *res0 = 0.f;
    if (nb == 0.0) {
        launch_fill_f64(s, ne, 0.0, x);
        return true;
    }
    float *V = c->gm_V.as<float>();
    for (int outer = 0; outer <= c->gm_refine; ++outer) {
        launch_gm_residual(s, ne, c->T0raw.as<double>(), x, b, c->gm_r.as<double>(), c->gm_nrm.as<double>(),
                           c->gm_host + 1);
        hip_check(hipStreamSynchronize(s), "GMRES");
        const double beta = std::sqrt(hv[1]);
        if (outer == 0) *res0 = (float)(beta / nb);
        if (!std::isfinite(beta)) return false;
        if (beta <= c->gm_tol * nb) return true;
        if (outer == c->gm_refine) break;
        // FP32 inner solve of T_0 d = r to a relative reduction tau
        const double tau = std::max(0.5 * c->gm_tol * nb / beta, 1e-6);
        launch_gm_start(s, ne, m, c->gm_r.as<double>(), c->gm_nrm.as<double>(), V, c->gm_g.as<double>());
        launch_gm_clear(s, m, c->gm_h1.as<double>(), c->gm_h2.as<double>(), c->gm_nrm.as<double>());
        // the previous solve's count for this pass, less one, runs without
        // waiting for the residual estimate (more iterations only lower it)
        const int p = outer < (int)c->gm_pred.size() ? std::max(0, c->gm_pred[outer] - 1) : 0;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            float *w = c->gm_w.as<float>();
            // h1, h2 and the norm accumulator are zero here (k_gm_clear, then
            // each Givens step clears what it read)
            launch_gm_matvec(s, ne, c->T0f.as<float>(), ld, V + (int64_t)j * ld, w);
            launch_gm_dots(s, ne, j + 1, V, ld, w, c->gm_h1.as<double>());
            launch_gm_update(s, ne, j + 1, V, ld, c->gm_h1.as<double>(), w, nullptr);
            launch_gm_dots(s, ne, j + 1, V, ld, w, c->gm_h2.as<double>());
            launch_gm_update(s, ne, j + 1, V, ld, c->gm_h2.as<double>(), w, c->gm_nrm.as<double>());
            launch_gm_givens(s, j, m, c->gm_h1.as<double>(), c->gm_h2.as<double>(), c->gm_nrm.as<double>(),
                             c->gm_R.as<double>(), c->gm_cs.as<double>(), c->gm_sn.as<double>(), c->gm_g.as<double>(),
                             c->gm_inv.as<double>(), c->gm_host);
            launch_gm_scale(s, ne, w, c->gm_inv.as<double>(), V + (int64_t)(j + 1) * ld);
            *iters += 1;
            k = j + 1;
            if (k < p) continue;
            hip_check(hipStreamSynchronize(s), "GMRES");
            const double res = hv[0];
            if (!(res > tau * beta)) break;
        }
        if (outer < (int)c->gm_pred.size()) c->gm_pred[outer] = k;
        launch_gm_solution(s, ne, k, m, c->gm_R.as<double>(), c->gm_g.as<double>(), c->gm_y.as<double>(), V, ld, x);
        c->gm_refines += 1;
    }
    return false;
}

}  // namespace qhp

extern "C" int qhp_set_gmres(qhp_ctx *ctx, double tol, int32_t m_max, int32_t max_refine, int32_t warm)
{
    QHP_ALLOC_SCOPE(ctx);
    if (!ctx) return QHP_EINVAL;
    if (!(tol > 0.0) || m_max < 1 || m_max > 512 || max_refine < 1 || warm < QHP_WARM_COLD || warm > QHP_WARM_BEST)
        return guard(ctx, QHP_EINVAL, "bad GMRES parameters");
    if (ctx->state < 2) return guard(ctx, QHP_ESTATE, "assemble first");
    if (ctx->state == 3 && ctx->nrhs != 1) return guard(ctx, QHP_EINVAL, "GMRES takes one right-hand side");
    if ((warm == QHP_WARM_MLP || warm == QHP_WARM_BEST) && !ctx->mlp)
        return guard(ctx, QHP_ESTATE, "attach a perceptron first");
    try {
        hip_check(hipSetDevice(ctx->p.device), "hipSetDevice");
        ctx->gm_tol = tol;
        ctx->gm_m = m_max;
        ctx->gm_refine = max_refine;
        ctx->gm_pred.assign(max_refine + 1, 0);
        ctx->warm = warm;
        qhp::gmres_prepare(ctx);
        ctx->p.solver = QHP_SOLVE_GMRES;
    } catch (const Fail &f) {
        return guard(ctx, f.code, f.msg);
    }
    return QHP_OK;
}

extern "C" int qhp_gmres_stats(const qhp_ctx *ctx, qhp_gmres_info *info, int32_t *iters, float *res0, int64_t n)
{
    if (!ctx || !info) return QHP_EINVAL;
    std::memset(info, 0, sizeof(*info));
    const int64_t ns = (int64_t)ctx->gm_iters.size();
    info->steps = ns;
    for (int64_t i = 0; i < ns; ++i) {
        info->iterations += ctx->gm_iters[i];
        info->max_iterations = std::max<int64_t>(info->max_iterations, ctx->gm_iters[i]);
    }
    info->refinements = ctx->gm_refines;
    info->fallbacks = ctx->gm_fallbacks;
    info->network_starts = ctx->gm_net_starts;
    for (int64_t i = 0; i < n && i < ns; ++i) {
        if (iters) iters[i] = ctx->gm_iters[i];
        if (res0) res0[i] = ctx->gm_res0[i];
    }
    return QHP_OK;
}

extern "C" int qhp_gmres_reset(qhp_ctx *ctx)
{
    QHP_ALLOC_SCOPE(ctx);
    if (!ctx) return QHP_EINVAL;
    ctx->gm_iters.clear();
    ctx->gm_res0.clear();
    ctx->gm_refines = 0;
    ctx->gm_fallbacks = 0;
    ctx->gm_net_starts = 0;
    return QHP_OK;
}
