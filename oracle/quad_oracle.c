/*
 * Plain C quadrature core of the CPU FP64 oracle.  TEST INFRASTRUCTURE ONLY:
 * called from the oracle Python modules through ctypes, never linked into the product.
 *
 * What it integrates (normalised units c = 1, eta = 1; every kernel carries
 * the 1/(4 pi) of the Green function):
 *   - retarded shell moments on the coarse mesh (Sec. II-A operators T^s, T^h
 *     tested with RWGs, Sec. II-C):
 *       V_j[m][n]   = int int_{shell j} f_m(r).f_n(r') / (4 pi R)
 *       S_j^p[c][c'] = int_c int_c'_{shell j} x^p / (4 pi R),  x = R/dt - j
 *   - retarded shell moments of the MFIE operator K tested with BC functions:
 *       N_j[m][n]   = int int_{shell j} g_m(r).((r - r') x f_n(r')) / (4 pi R^3)
 *   - the Yukawa matrices of Sec. II-C (wave number -j kappa):
 *       Zs[m][n] = int int g_m.g_n e^{-kR}/(4 pi R)   (BC-BC)
 *       D[v][v'] = sum over fine pairs in the dual cells of v, v' of
 *                  int int e^{-kR}/(4 pi R) / (A_t A_t')
 *       M[m][n]  = int int g_m.((r - r') x f_n) (1 + kR) e^{-kR} / (4 pi R^3)
 *   where shell j is the distance range j dt < R <= (j+1) dt.
 *
 * Inner (source) integrals use polar coordinates about the projection p of
 * the test point on the source plane: the triangle is the signed sum of the
 * three triangles (p, a_i, a_i+1); on each, the radial integral is done in
 * closed form in R (R dR = rho drho) and the angle by Gauss-Legendre in
 * s = asinh(t/h) (t along the edge, h the distance of p to the edge line;
 * dpsi = ds/cosh s) on every sub-interval between the points where a shell
 * circle crosses the edge; where the shell lies wholly inside the edge's
 * wedge the radial pieces are constant and the angular integrals exact.  Outer (test) integrals use the symmetric rule passed in.
 *
 * The RT0 representation: on a triangle with vertices P0,P1,P2 and area A a
 * field with outward fluxes F0,F1,F2 (through the edges opposite P0,P1,P2) is
 * sum_i F_i (r - P_i)/(2A).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define FOUR_PI (4.0 * 3.14159265358979323846)

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }

/* output of one inner integral; x = R/dt - j on shell j */
typedef struct {
    double I0;      /* int 1/R                          */
    double Iu[3];   /* int (r' - p)/R                   */
    double Sx[4];   /* int x^a / R, a = 0..3            */
    double W[3];    /* int (r - r')/R^3                 */
    double I0x[2];  /* int x^a / R, a = 1, 2 (= Sx)     */
    double Iux[3];  /* int x (r' - p)/R                 */
    double Wx[2][3]; /* int x^a (r - r')/R^3, a = 1, 2  */
} inner_t;

/* closed-form radial pieces between R = lo and R = hi (lo >= |d|) */
/* radial pieces between R = lo and R = hi (lo >= |d|) of the kernels over
   the source plane (R dR = rho drho), x = R/dt - j running from xoff_lo to
   xoff_hi:
     P0  = int dR,  P1 = int rho dR,  X[a] = int x^a dR (a = 0..3)
     dQ0 = d int dR/R^2,  Q1 = int rho/R^2 dR
     P1x = int x rho dR;  dQx[a-1] = d int x^a/R^2 dR,  Qx[a-1] = int x^a rho/R^2 dR
   (a = 1, 2), from x = R/dt - j and the antiderivatives of rho = sqrt(R^2 - d^2)
   times 1, R, 1/R, 1/R^2: P1, rho^3/3, rho - |d| acos(|d|/R), Q1 */
typedef struct {
    double P0, P1, X[4], dQ0, Q1, P1x, dQx[2], Qx[2];
} radial_t;

static void radial(double lo, double hi, double d, double xoff_lo, double xoff_hi, double dt,
                   int lo_is_plane, double jsh, radial_t *o)
{
    double d2 = d * d, ad = fabs(d);
    double slo = sqrt(fmax(lo * lo - d2, 0.0));
    double shi = sqrt(fmax(hi * hi - d2, 0.0));
    o->P0 = hi - lo;
    double lg = 0.0;
    if (d2 > 0.0 && lo + slo > 0.0) lg = log((hi + shi) / (lo + slo));
    o->P1 = 0.5 * (hi * shi - lo * slo) - 0.5 * d2 * lg;
    double xl = xoff_lo, xh = xoff_hi;
    o->X[0] = dt * (xh - xl);
    o->X[1] = dt * (xh * xh - xl * xl) / 2.0;
    o->X[2] = dt * (xh * xh * xh - xl * xl * xl) / 3.0;
    o->X[3] = dt * (xh * xh * xh * xh - xl * xl * xl * xl) / 4.0;
    /* d * int dR/R^2 and int sqrt(R^2-d^2)/R^2 dR */
    if (lo_is_plane) {
        o->dQ0 = (d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0)) - d / hi;
        double lnlo = (lo > 0.0) ? log(lo) : 0.0; /* s_lo = 0 at R = |d| */
        o->Q1 = -shi / hi + log(hi + shi) - lnlo;
    } else {
        o->dQ0 = d / lo - d / hi;
        o->Q1 = -shi / hi + slo / lo + log((hi + shi) / (lo + slo));
    }
    /* x-weighted pieces (only where lo > 0: the plane's own shell starts at |d|) */
    double inv = 1.0 / dt;
    o->P1x = inv * (shi * shi * shi - slo * slo * slo) / 3.0 - jsh * o->P1;
    double flog = (lo > 0.0) ? log(hi / lo) : 0.0;
    double acl = (lo > 0.0) ? acos(fmin(1.0, ad / lo)) : 0.0, ach = acos(fmin(1.0, ad / hi));
    double G1 = (shi - ad * ach) - (slo - ad * acl); /* int sqrt(R^2-d^2)/R dR */
    o->dQx[0] = d * inv * flog - jsh * o->dQ0;
    o->Qx[0] = inv * G1 - jsh * o->Q1;
    o->dQx[1] = d * inv * inv * (hi - lo) - 2.0 * jsh * d * inv * flog + jsh * jsh * o->dQ0;
    o->Qx[1] = inv * inv * o->P1 - 2.0 * jsh * inv * G1 + jsh * jsh * o->Q1;
}

static void sort_small(double *a, int n)
{
    for (int i = 1; i < n; ++i) {
        double v = a[i];
        int k = i - 1;
        while (k >= 0 && a[k] > v) { a[k + 1] = a[k]; --k; }
        a[k + 1] = v;
    }
}

/* add one radial piece: ws the angle weight, wv the angle-weighted in-plane
   radial direction */
static void accumulate(inner_t *out, const radial_t *o, double ws, const double *wv, const double *nrm,
                       int coplanar)
{
    out->I0 += ws * o->P0;
    for (int k = 0; k < 3; ++k) out->Iu[k] += o->P1 * wv[k];
    for (int a = 0; a < 4; ++a) out->Sx[a] += ws * o->X[a];
    for (int a = 0; a < 2; ++a) out->I0x[a] += ws * o->X[a + 1];
    for (int k = 0; k < 3; ++k) out->Iux[k] += o->P1x * wv[k];
    if (!coplanar) {
        for (int k = 0; k < 3; ++k) out->W[k] += ws * o->dQ0 * nrm[k] - o->Q1 * wv[k];
        for (int a = 0; a < 2; ++a)
            for (int k = 0; k < 3; ++k) out->Wx[a][k] += ws * o->dQx[a] * nrm[k] - o->Qx[a] * wv[k];
    }
}

/*
 * Integral over triangle P (vertices P[0..2], counter-clockwise about its
 * normal) from test point r, restricted to s_lo < R <= s_hi.
 */
static void inner_integral(const double P[3][3], const double *r, double s_lo, double s_hi,
                           double jsh, double dt, int ng, const double *gx, const double *gw,
                           double coplanar_tol, inner_t *out)
{
    memset(out, 0, sizeof(*out));
    double e1[3], e2[3], nrm[3];
    for (int k = 0; k < 3; ++k) { e1[k] = P[1][k] - P[0][k]; e2[k] = P[2][k] - P[0][k]; }
    cross3(e1, e2, nrm);
    double nn = norm3(nrm);
    for (int k = 0; k < 3; ++k) nrm[k] /= nn;
    double rp0[3];
    for (int k = 0; k < 3; ++k) rp0[k] = r[k] - P[0][k];
    double d = dot3(rp0, nrm);
    double ad = fabs(d);
    double p[3];
    for (int k = 0; k < 3; ++k) p[k] = r[k] - d * nrm[k];
    double lmax = fmax(norm3(e1), norm3(e2));
    int coplanar = ad <= coplanar_tol * lmax;
    double R_lo = fmax(s_lo, ad);
    int lo_is_plane = !(s_lo > ad);
    if (!(s_hi > R_lo)) return;

    for (int i = 0; i < 3; ++i) {
        const double *a = P[i], *b = P[(i + 1) % 3];
        double et[3], len = 0.0;
        for (int k = 0; k < 3; ++k) et[k] = b[k] - a[k];
        len = norm3(et);
        for (int k = 0; k < 3; ++k) et[k] /= len;
        double ap[3];
        for (int k = 0; k < 3; ++k) ap[k] = a[k] - p[k];
        double ta = dot3(ap, et);
        double tb = ta + len;
        double wh[3];
        for (int k = 0; k < 3; ++k) wh[k] = ap[k] - ta * et[k];
        double h = norm3(wh);
        if (h <= 1e-12 * len) continue; /* degenerate sub-triangle */
        double eh[3];
        for (int k = 0; k < 3; ++k) eh[k] = wh[k] / h;
        double c3[3];
        cross3(eh, et, c3);
        double sig = dot3(c3, nrm) > 0.0 ? 1.0 : -1.0;
        /* angular variable along the edge: s = asinh(t/h), t the coordinate
           along the edge from the foot of p; dpsi = ds / cosh(s) */
        double pa = asinh(ta / h), pb = asinh(tb / h);
        /* break points where a segment circle crosses the edge line */
        double brk[6];
        int nb = 0;
        brk[nb++] = pa;
        double hd2 = h * h + d * d;
        double Rs[2] = {s_lo, s_hi};
        for (int q = 0; q < 2; ++q) {
            double Rq = Rs[q];
            if (isinf(Rq) || !(Rq * Rq > hd2)) continue;
            double ts = sqrt(Rq * Rq - hd2);
            double ps = asinh(ts / h);
            if (-ps > pa && -ps < pb) brk[nb++] = -ps;
            if (ps > pa && ps < pb) brk[nb++] = ps;
        }
        brk[nb++] = pb;
        sort_small(brk, nb);
        for (int s = 0; s + 1 < nb; ++s) {
            double lo = brk[s], hi = brk[s + 1];
            if (!(hi > lo)) continue;
            double mid = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
            double cm = cosh(mid);
            double Rm = sqrt(h * h * cm * cm + d * d);
            if (!(Rm > R_lo)) continue; /* segment empty on this interval */
            if (Rm >= s_hi) {
                /* the whole shell lies inside the edge's wedge here: the radial
                   pieces are constants and the angular integrals are exact */
                radial_t o;
                radial(R_lo, s_hi, d, R_lo / dt - jsh, s_hi / dt - jsh, dt, lo_is_plane, jsh, &o);
                double dpsi = atan(sinh(hi)) - atan(sinh(lo));
                double cu = tanh(hi) - tanh(lo);           /* int sin(psi) dpsi ... */
                double su = 1.0 / cosh(hi) - 1.0 / cosh(lo); /* ... and -int cos(psi) */
                double du[3];
                for (int k = 0; k < 3; ++k) du[k] = sig * (cu * eh[k] - su * et[k]);
                accumulate(out, &o, sig * dpsi, du, nrm, coplanar);
                continue;
            }
            for (int g = 0; g < ng; ++g) {
                double sv = mid + half * gx[g];
                double ch = cosh(sv), sh = sinh(sv);
                double Rhi = sqrt(h * h * ch * ch + d * d);
                double wgt = sig * half * gw[g] / ch;
                double u[3];
                for (int k = 0; k < 3; ++k) u[k] = (eh[k] + sh * et[k]) / ch;
                radial_t o;
                radial(R_lo, Rhi, d, R_lo / dt - jsh, Rhi / dt - jsh, dt, lo_is_plane, jsh, &o);
                double wu[3];
                for (int k = 0; k < 3; ++k) wu[k] = wgt * u[k];
                accumulate(out, &o, wgt, wu, nrm, coplanar);
            }
        }
    }
}

/* Python-callable single inner integral (used by the oracle's pins). */
void orc_inner(const double *P, const double *r, double s_lo, double s_hi, double jsh, double dt,
               int ng, const double *gx, const double *gw, double coplanar_tol, double *out10)
{
    double PP[3][3];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) PP[i][k] = P[3 * i + k];
    inner_t o;
    inner_integral(PP, r, s_lo, s_hi, jsh, dt, ng, gx, gw, coplanar_tol, &o);
    out10[0] = o.I0;
    for (int k = 0; k < 3; ++k) {
        out10[1 + k] = o.Iu[k];
        out10[4 + k] = o.Sx[k];
        out10[7 + k] = o.W[k];
    }
}

/* the x-weighted moments of one inner integral (pins of the higher-order
   temporal bases): out13 = Sx[3], Iux[0..2], Wx[0][0..2], Wx[1][0..2] */
void orc_inner_x(const double *P, const double *r, double s_lo, double s_hi, double jsh, double dt,
                 int ng, const double *gx, const double *gw, double coplanar_tol, double *out13)
{
    double PP[3][3];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) PP[i][k] = P[3 * i + k];
    inner_t o;
    inner_integral(PP, r, s_lo, s_hi, jsh, dt, ng, gx, gw, coplanar_tol, &o);
    out13[0] = o.Sx[3];
    for (int k = 0; k < 3; ++k) {
        out13[1 + k] = o.Iux[k];
        out13[4 + k] = o.Wx[0][k];
        out13[7 + k] = o.Wx[1][k];
    }
    out13[10] = o.I0x[0];
    out13[11] = o.I0x[1];
    out13[12] = 0.0;
}

static void load_tri(const double *xyz, const long *tri, long c, double P[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) P[i][k] = xyz[3 * tri[3 * c + i] + k];
}

static double tri_area(const double P[3][3])
{
    double e1[3], e2[3], c[3];
    for (int k = 0; k < 3; ++k) { e1[k] = P[1][k] - P[0][k]; e2[k] = P[2][k] - P[0][k]; }
    cross3(e1, e2, c);
    return 0.5 * norm3(c);
}

/* smallest and largest distance from r to triangle P */
static void dist_range(const double P[3][3], const double *r, double *dmin, double *dmax)
{
    double mx = 0.0;
    for (int i = 0; i < 3; ++i) {
        double v[3];
        for (int k = 0; k < 3; ++k) v[k] = P[i][k] - r[k];
        mx = fmax(mx, norm3(v));
    }
    /* point-triangle distance via projection and edge distances */
    double e1[3], e2[3], n[3];
    for (int k = 0; k < 3; ++k) { e1[k] = P[1][k] - P[0][k]; e2[k] = P[2][k] - P[0][k]; }
    cross3(e1, e2, n);
    double nn = norm3(n);
    for (int k = 0; k < 3; ++k) n[k] /= nn;
    double rp[3];
    for (int k = 0; k < 3; ++k) rp[k] = r[k] - P[0][k];
    double d = dot3(rp, n);
    double q[3];
    for (int k = 0; k < 3; ++k) q[k] = r[k] - d * n[k];
    int inside = 1;
    for (int i = 0; i < 3; ++i) {
        const double *a = P[i], *b = P[(i + 1) % 3];
        double ab[3], aq[3], c[3];
        for (int k = 0; k < 3; ++k) { ab[k] = b[k] - a[k]; aq[k] = q[k] - a[k]; }
        cross3(ab, aq, c);
        if (dot3(c, n) < 0.0) inside = 0;
    }
    double best;
    if (inside) {
        best = fabs(d);
    } else {
        best = 1e300;
        for (int i = 0; i < 3; ++i) {
            const double *a = P[i], *b = P[(i + 1) % 3];
            double ab[3], ar[3];
            for (int k = 0; k < 3; ++k) { ab[k] = b[k] - a[k]; ar[k] = r[k] - a[k]; }
            double t = dot3(ar, ab) / dot3(ab, ab);
            t = fmin(1.0, fmax(0.0, t));
            double v[3];
            for (int k = 0; k < 3; ++k) v[k] = r[k] - (a[k] + t * ab[k]);
            best = fmin(best, norm3(v));
        }
    }
    *dmin = best;
    *dmax = mx;
}

static void shell_range(double dmin, double dmax, double dt, long n_shells, long *j0, long *j1)
{
    long a = (long)floor(dmin / dt) - 1;
    long b = (long)floor(dmax / dt);
    if (a < 0) a = 0;
    if (b > n_shells - 1) b = n_shells - 1;
    *j0 = a;
    *j1 = b;
}

/*
 * Retarded coarse-coarse shell moments for temporal bases of order `order`
 * (1 or 2):
 *   V  [n_shells][order][ne][ne]   x^a weights, a < order (accumulated, not symmetrised)
 *   S  [n_shells][order + 2][nc][nc]   a <= order + 1
 */
void orc_retarded_coarse(const double *xyz, const long *tri, long nc, const long *tri_edge,
                         const long *tri_sign, long ne, double dt, long n_shells, int order, int nq,
                         const double *qbary, const double *qw, int ng, const double *gx,
                         const double *gw, double *V, double *S)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (long c = 0; c < nc; ++c) {
        double P[3][3];
        load_tri(xyz, tri, c, P);
        double A = tri_area(P);
        for (long cs = 0; cs < nc; ++cs) {
            double Q[3][3];
            load_tri(xyz, tri, cs, Q);
            double As = tri_area(Q);
            for (int q = 0; q < nq; ++q) {
                double r[3];
                for (int k = 0; k < 3; ++k)
                    r[k] = qbary[3 * q] * P[0][k] + qbary[3 * q + 1] * P[1][k] + qbary[3 * q + 2] * P[2][k];
                double wq = qw[q] * A;
                double dmin, dmax;
                dist_range(Q, r, &dmin, &dmax);
                long j0, j1;
                shell_range(dmin, dmax, dt, n_shells, &j0, &j1);
                /* projection point of r on the source plane (for I_u) */
                double e1[3], e2[3], n[3];
                for (int k = 0; k < 3; ++k) { e1[k] = Q[1][k] - Q[0][k]; e2[k] = Q[2][k] - Q[0][k]; }
                cross3(e1, e2, n);
                double nn = norm3(n);
                for (int k = 0; k < 3; ++k) n[k] /= nn;
                double rq0[3];
                for (int k = 0; k < 3; ++k) rq0[k] = r[k] - Q[0][k];
                double dd = dot3(rq0, n);
                double pp[3];
                for (int k = 0; k < 3; ++k) pp[k] = r[k] - dd * n[k];
                for (long j = j0; j <= j1; ++j) {
                    inner_t o;
                    inner_integral(Q, r, j * dt, (j + 1) * dt, (double)j, dt, ng, gx, gw, 1e-12, &o);
                    for (int p = 0; p < order + 2; ++p) {
                        double val = wq * o.Sx[p] / FOUR_PI;
#pragma omp atomic
                        S[((j * (order + 2) + p) * nc + c) * nc + cs] += val;
                    }
                    for (int a = 0; a < 3; ++a) {
                        long m = tri_edge[3 * c + a];
                        double fa[3];
                        for (int k = 0; k < 3; ++k) fa[k] = tri_sign[3 * c + a] * (r[k] - P[a][k]) / (2.0 * A);
                        for (int b = 0; b < 3; ++b) {
                            long nidx = tri_edge[3 * cs + b];
                            for (int xa = 0; xa < order; ++xa) {
                                const double *iu = xa == 0 ? o.Iu : o.Iux;
                                double i0 = xa == 0 ? o.I0 : o.I0x[0];
                                double vb[3];
                                for (int k = 0; k < 3; ++k) vb[k] = iu[k] + (pp[k] - Q[b][k]) * i0;
                                double val = wq * tri_sign[3 * cs + b] / (2.0 * As) * dot3(fa, vb) / FOUR_PI;
#pragma omp atomic
                                V[((j * order + xa) * ne + m) * ne + nidx] += val;
                            }
                        }
                    }
                }
            }
        }
    }
}

/* BC field on fine triangle t at r, from its outward fluxes */
static void rt0_eval(const double P[3][3], double A, const double *F, const double *r, double *out)
{
    for (int k = 0; k < 3; ++k) out[k] = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) out[k] += F[i] * (r[k] - P[i][k]) / (2.0 * A);
}

/*
 * Retarded BC-RWG shell moments of the MFIE kernel for temporal bases of
 * order `order` (1 or 2):
 *   N [n_shells][order + 1][ne][ne]   x^a weights, a <= order
 * bc_off[t]..bc_off[t+1] index bc_edge / bc_flux (3 per entry) for fine t.
 */
void orc_retarded_bc(const double *fxyz, const long *ftri, long nf, const long *fparent,
                     const long *bc_off, const long *bc_edge, const double *bc_flux,
                     const double *xyz, const long *tri, long nc, const long *tri_edge,
                     const long *tri_sign, long ne, double dt, long n_shells, int order, int nq,
                     const double *qbary, const double *qw, int ng, const double *gx,
                     const double *gw, double coplanar_tol, double *N)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < nf; ++t) {
        double P[3][3];
        load_tri(fxyz, ftri, t, P);
        double A = tri_area(P);
        for (long cs = 0; cs < nc; ++cs) {
            if (fparent[t] == cs) continue; /* coplanar: integrand is zero */
            double Q[3][3];
            load_tri(xyz, tri, cs, Q);
            double As = tri_area(Q);
            for (int q = 0; q < nq; ++q) {
                double r[3];
                for (int k = 0; k < 3; ++k)
                    r[k] = qbary[3 * q] * P[0][k] + qbary[3 * q + 1] * P[1][k] + qbary[3 * q + 2] * P[2][k];
                double wq = qw[q] * A;
                double dmin, dmax;
                dist_range(Q, r, &dmin, &dmax);
                long j0, j1;
                shell_range(dmin, dmax, dt, n_shells, &j0, &j1);
                for (long j = j0; j <= j1; ++j) {
                    inner_t o;
                    inner_integral(Q, r, j * dt, (j + 1) * dt, (double)j, dt, ng, gx, gw, coplanar_tol, &o);
                    for (int b = 0; b < 3; ++b) {
                        long nidx = tri_edge[3 * cs + b];
                        double rb[3];
                        for (int k = 0; k < 3; ++k) rb[k] = r[k] - Q[b][k];
                        double sb = tri_sign[3 * cs + b] / (2.0 * As);
                        for (int xa = 0; xa <= order; ++xa) {
                            double wx[3];
                            cross3(xa == 0 ? o.W : o.Wx[xa - 1], rb, wx);
                            for (long e = bc_off[t]; e < bc_off[t + 1]; ++e) {
                                double g[3];
                                rt0_eval(P, A, bc_flux + 3 * e, r, g);
                                double val = wq * sb * dot3(wx, g) / FOUR_PI;
#pragma omp atomic
                                N[((j * (order + 1) + xa) * ne + bc_edge[e]) * ne + nidx] += val;
                            }
                        }
                    }
                }
            }
        }
    }
}

static int share_vertex(const long *tri, long c1, long c2)
{
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k)
            if (tri[3 * c1 + i] == tri[3 * c2 + k]) return 1;
    return 0;
}

/* e^{-x} - 1 over x, times -1 at x = 0 handled by expm1 */
static double yuk_rem(double R, double kappa)
{
    double x = kappa * R;
    if (x == 0.0) return -kappa / FOUR_PI;
    return expm1(-x) / R / FOUR_PI;
}

/* ((1 + x) e^{-x} - 1) / x^2 */
static double mf_phi(double x)
{
    if (x < 0.1) {
        /* series: -1/2 + x/3 - x^2/8 + x^3/30 - x^4/144 + x^5/840 - x^6/5760 + x^7/45360 */
        double c[8] = {-1.0 / 2.0, 1.0 / 3.0, -1.0 / 8.0, 1.0 / 30.0, -1.0 / 144.0, 1.0 / 840.0,
                       -1.0 / 5760.0, 1.0 / 45360.0};
        double s = 0.0, xp = 1.0;
        for (int i = 0; i < 8; ++i) { s += c[i] * xp; xp *= x; }
        return s;
    }
    return ((1.0 + x) * exp(-x) - 1.0) / (x * x);
}

/*
 * Static Yukawa BC-BC operators on the fine mesh.
 *   Zs [ne][ne] = int int g_m . g_n e^{-kR}/(4 pi R)
 *   D  [nv][nv] = sum_{t in C(v), t' in C(v')} int int e^{-kR}/(4 pi R) / (A_t A_t')
 */
void orc_static_bcbc(const double *fxyz, const long *ftri, long nf, const long *fparent,
                     const long *fowner, const long *tri, const long *bc_off, const long *bc_edge,
                     const double *bc_flux, long ne, long nv, double kappa, int nq,
                     const double *qbary, const double *qw, int ns, const double *sbary,
                     const double *sw, int ng, const double *gx, const double *gw, double *Zs,
                     double *D)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < nf; ++t) {
        double P[3][3];
        load_tri(fxyz, ftri, t, P);
        double A = tri_area(P);
        for (long ts = 0; ts < nf; ++ts) {
            double Q[3][3];
            load_tri(fxyz, ftri, ts, Q);
            double As = tri_area(Q);
            int near = share_vertex(tri, fparent[t], fparent[ts]);
            /* local matrix Mab = int int Phi_a . Phi'_b G, scalar J = int int G */
            double M[3][3] = {{0}}, J = 0.0;
            for (int q = 0; q < nq; ++q) {
                double r[3];
                for (int k = 0; k < 3; ++k)
                    r[k] = qbary[3 * q] * P[0][k] + qbary[3 * q + 1] * P[1][k] + qbary[3 * q + 2] * P[2][k];
                double wq = qw[q] * A;
                /* inner vectors Vb = int (r' - Q_b) G ds', scalar I = int G ds' */
                double Vb[3][3] = {{0}}, I = 0.0;
                if (near) {
                    inner_t o;
                    inner_integral(Q, r, 0.0, INFINITY, 0.0, 1.0, ng, gx, gw, 1e-12, &o);
                    double e1[3], e2[3], n[3];
                    for (int k = 0; k < 3; ++k) { e1[k] = Q[1][k] - Q[0][k]; e2[k] = Q[2][k] - Q[0][k]; }
                    cross3(e1, e2, n);
                    double nn = norm3(n);
                    for (int k = 0; k < 3; ++k) n[k] /= nn;
                    double rq0[3];
                    for (int k = 0; k < 3; ++k) rq0[k] = r[k] - Q[0][k];
                    double dd = dot3(rq0, n);
                    I += o.I0 / FOUR_PI;
                    for (int b = 0; b < 3; ++b)
                        for (int k = 0; k < 3; ++k)
                            Vb[b][k] += (o.Iu[k] + (r[k] - dd * n[k] - Q[b][k]) * o.I0) / FOUR_PI;
                }
                for (int s = 0; s < ns; ++s) {
                    double rs[3], dr[3];
                    for (int k = 0; k < 3; ++k) {
                        rs[k] = sbary[3 * s] * Q[0][k] + sbary[3 * s + 1] * Q[1][k] + sbary[3 * s + 2] * Q[2][k];
                        dr[k] = r[k] - rs[k];
                    }
                    double R = norm3(dr);
                    double G = near ? yuk_rem(R, kappa) : exp(-kappa * R) / (FOUR_PI * R);
                    double ws = sw[s] * As;
                    I += ws * G;
                    for (int b = 0; b < 3; ++b)
                        for (int k = 0; k < 3; ++k) Vb[b][k] += ws * (rs[k] - Q[b][k]) * G;
                }
                J += wq * I;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        double s = 0.0;
                        for (int k = 0; k < 3; ++k) s += (r[k] - P[a][k]) * Vb[b][k];
                        M[a][b] += wq * s / (4.0 * A * As);
                    }
            }
            for (long e = bc_off[t]; e < bc_off[t + 1]; ++e) {
                const double *F = bc_flux + 3 * e;
                for (long es = bc_off[ts]; es < bc_off[ts + 1]; ++es) {
                    const double *Fs = bc_flux + 3 * es;
                    double s = 0.0;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) s += F[a] * M[a][b] * Fs[b];
#pragma omp atomic
                    Zs[bc_edge[e] * ne + bc_edge[es]] += s;
                }
            }
#pragma omp atomic
            D[fowner[t] * nv + fowner[ts]] += J / (A * As);
        }
    }
}

/*
 * Static Yukawa MFIE matrix, BC test (fine) x RWG trial (coarse).
 *   M [ne][ne] = int int g_m . ((r - r') x f_n) (1 + kR) e^{-kR} / (4 pi R^3)
 */
void orc_static_mfie(const double *fxyz, const long *ftri, long nf, const long *fparent,
                     const long *bc_off, const long *bc_edge, const double *bc_flux,
                     const double *xyz, const long *tri, long nc, const long *tri_edge,
                     const long *tri_sign, long ne, double kappa, int nq, const double *qbary,
                     const double *qw, int ns, const double *sbary, const double *sw, int ng,
                     const double *gx, const double *gw, double coplanar_tol, double *M)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < nf; ++t) {
        double P[3][3];
        load_tri(fxyz, ftri, t, P);
        double A = tri_area(P);
        for (long cs = 0; cs < nc; ++cs) {
            if (fparent[t] == cs) continue;
            double Q[3][3];
            load_tri(xyz, tri, cs, Q);
            double As = tri_area(Q);
            int near = share_vertex(tri, fparent[t], cs);
            for (int q = 0; q < nq; ++q) {
                double r[3];
                for (int k = 0; k < 3; ++k)
                    r[k] = qbary[3 * q] * P[0][k] + qbary[3 * q + 1] * P[1][k] + qbary[3 * q + 2] * P[2][k];
                double wq = qw[q] * A;
                /* W = int (r - r') K(R) / (4 pi) ds' with K = (1+kR)e^{-kR}/R^3 */
                double W[3] = {0, 0, 0};
                if (near) {
                    inner_t o;
                    inner_integral(Q, r, 0.0, INFINITY, 0.0, 1.0, ng, gx, gw, coplanar_tol, &o);
                    for (int k = 0; k < 3; ++k) W[k] += o.W[k] / FOUR_PI;
                }
                for (int s = 0; s < ns; ++s) {
                    double rs[3], dr[3];
                    for (int k = 0; k < 3; ++k) {
                        rs[k] = sbary[3 * s] * Q[0][k] + sbary[3 * s + 1] * Q[1][k] + sbary[3 * s + 2] * Q[2][k];
                        dr[k] = r[k] - rs[k];
                    }
                    double R = norm3(dr);
                    double x = kappa * R;
                    double K = near ? kappa * kappa * mf_phi(x) / R : (1.0 + x) * exp(-x) / (R * R * R);
                    double ws = sw[s] * As;
                    for (int k = 0; k < 3; ++k) W[k] += ws * dr[k] * K / FOUR_PI;
                }
                for (int b = 0; b < 3; ++b) {
                    long nidx = tri_edge[3 * cs + b];
                    double rb[3], wx[3];
                    for (int k = 0; k < 3; ++k) rb[k] = r[k] - Q[b][k];
                    cross3(W, rb, wx);
                    double sb = tri_sign[3 * cs + b] / (2.0 * As);
                    for (long e = bc_off[t]; e < bc_off[t + 1]; ++e) {
                        double g[3];
                        rt0_eval(P, A, bc_flux + 3 * e, r, g);
                        double val = wq * sb * dot3(wx, g);
#pragma omp atomic
                        M[bc_edge[e] * ne + nidx] += val;
                    }
                }
            }
        }
    }
}
