// Device-side mesh tables and the assembly kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qhp {

constexpr int kMaxValence = 12;  // largest vertex valence the BC kernels accept

// Device pointers to the mesh tables (see Mesh) plus quadrature scalars.
// up to 16 terms c[t] * p[t] of a lag combination (passed by value)
struct LinTerms {
    int n = 0;
    const double *p[16] = {};
    double c[16] = {};
    void add(const double *ptr, double coef)
    {
        if (ptr && coef != 0.0 && n < 16) {
            p[n] = ptr;
            c[n] = coef;
            ++n;
        }
    }
};

struct AsmArgs {
    int64_t nv, ne, nc, nf;
    const double *xyz;
    const int32_t *tri;
    const int32_t *edges;
    const int32_t *cells;
    const int32_t *tri_edge;
    const int32_t *tri_sign;
    const double *area;
    const int32_t *valence;
    const double *fxyz;
    const int32_t *ftri;
    const int32_t *fparent;
    const int32_t *fowner;
    const int32_t *bc_off;
    const int32_t *bc_edge;
    const int32_t *bc_local;
    const double *bc_flux;
    const int32_t *vcell_off;
    const int32_t *vcell_tri;
    const int32_t *vedge_off;
    const int32_t *vedge;
    // transposed BC table: entries of each BC function
    const int32_t *bct_off;
    const int32_t *bct_entry;
    const int32_t *bc_tri;
    double dt;
    double coplanar_tol;
    int ng;
};

void set_gauss(const double *x, const double *w, int n);
void launch_gram(hipStream_t s, const AsmArgs &g, double *G);
// shell moments for temporal bases of order 1 (hat functions) or 2
// (quadratic interpolators): V [shell][order][ne][ne], S [shell][order + 2][nc][nc],
// N [shell][order + 1][ne][ne] (x^a weights, x = R/dt - j)
void launch_ret_coarse(hipStream_t s, const AsmArgs &g, int order, int64_t j0, int64_t j1, double *V, double *S);
void launch_ret_bc(hipStream_t s, const AsmArgs &g, int order, int64_t j0, int64_t j1, double *N);
void launch_yuk_bcbc(hipStream_t s, const AsmArgs &g, double kappa, double *Zs, double *D);
void launch_yuk_mfie(hipStream_t s, const AsmArgs &g, double kappa, double *M);
void launch_laplacians(hipStream_t s, const AsmArgs &g, double *LS, double *LL);
void launch_sub_const(hipStream_t s, int64_t n, double *X);
void launch_proj(hipStream_t s, int64_t ne, const int32_t *pairs, const double *Lp, int64_t nl, double *P);
void launch_zh(hipStream_t s, const AsmArgs &g, double kappa, const double *D, double *Zh);
void launch_bk(hipStream_t s, const AsmArgs &g, const double *Sk, const double *Sk1, const double *Sk2,
               double T0, double *B);
void launch_sym_s(hipStream_t s, int64_t nc, int np, double *S);
// Sq_k [nc][nc]: the q_0 combination of the shell moments of lag k (Sec. IV-A)
void launch_sq(hipStream_t s, int64_t nc, const double *Sk, const double *Sk1, const double *Sk2, double *Sq);
void launch_lag_ac(hipStream_t s, int64_t nn, int64_t k, double dt, const double *Vk, const double *Vk1,
                   const double *Nk, const double *Nk1, const double *G, double *A, double *C);
void launch_lin3(hipStream_t s, int64_t n, double *X, double a, const double *Y, double b, const double *Z,
                 double c);

// out = base_c * base + sum of the terms (base may be null)
void launch_lincomb(hipStream_t s, int64_t n, const LinTerms &t, double base_c, const double *base, double *out);
// B_k = -T0 Sigma diag(1/A) Sq diag(1/A) Sigma^T from a formed Sq_k
void launch_bk_sq(hipStream_t s, const AsmArgs &g, const double *Sq, double T0, double *B);

}  // namespace qhp
