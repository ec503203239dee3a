// Quadrature assembly kernels (gfx950, FP64): Gram, Yukawa operators and the
// retarded shell moments from which the lag blocks are combined.
//
// Written quadrature specification (the paper states none):
//   * test integrals: Radon's 7-point degree-5 rule on coarse triangles, the
//     3-point degree-2 rule on fine (barycentric) triangles;
//   * source integrals of 1/R, x^p/R and (r-r')/R^3 on a distance shell
//     j dt < R <= (j+1) dt: polar coordinates about the projection p of the
//     test point on the source plane, closed forms in R (R dR = rho drho),
//     angular Gauss-Legendre in s = asinh(t/h) (t along an edge, h the distance
//     of p to its line) on each sub-interval between shell-circle crossings;
//     where the shell lies wholly inside an edge's wedge the angular integrals
//     are exact;
//   * Yukawa kernels: for fine pairs whose coarse parents share a vertex the
//     static part uses the polar scheme and the bounded remainder a 7-point
//     source rule; other pairs use the 7-point source rule for the whole kernel;
//   * MFIE-type kernels vanish for a fine test triangle inside the source
//     triangle and for test points within 1e-12 (source edge) of its plane.
// All kernels include the 1/(4 pi) of the Green function.
#include "assembly.h"

namespace qhp {

__constant__ double c_gx[32];
__constant__ double c_gw[32];

static const double kFourPi = 12.566370614359172953850573533118;

// Radon 7-point rule, barycentric coordinates, and the 3-point rule
__device__ __forceinline__ void radon7_point(int q, double &l0, double &l1, double &l2, double &w)
{
    const double s15 = 3.872983346207416885179265399782;
    const double a1 = (9.0 - 2.0 * s15) / 21.0, b1 = (6.0 + s15) / 21.0;
    const double a2 = (9.0 + 2.0 * s15) / 21.0, b2 = (6.0 - s15) / 21.0;
    const double w1 = (155.0 + s15) / 1200.0, w2 = (155.0 - s15) / 1200.0;
    switch (q) {
    case 0: l0 = l1 = l2 = 1.0 / 3.0; w = 9.0 / 40.0; break;
    case 1: l0 = a1; l1 = b1; l2 = b1; w = w1; break;
    case 2: l0 = b1; l1 = a1; l2 = b1; w = w1; break;
    case 3: l0 = b1; l1 = b1; l2 = a1; w = w1; break;
    case 4: l0 = a2; l1 = b2; l2 = b2; w = w2; break;
    case 5: l0 = b2; l1 = a2; l2 = b2; w = w2; break;
    default: l0 = b2; l1 = b2; l2 = a2; w = w2; break;
    }
}
__device__ __forceinline__ void tri3_point(int q, double &l0, double &l1, double &l2, double &w)
{
    l0 = (q == 0) ? 2.0 / 3.0 : 1.0 / 6.0;
    l1 = (q == 1) ? 2.0 / 3.0 : 1.0 / 6.0;
    l2 = (q == 2) ? 2.0 / 3.0 : 1.0 / 6.0;
    w = 1.0 / 3.0;
}

struct V3 {
    double x, y, z;
};
__device__ __forceinline__ V3 mk(double x, double y, double z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator*(double s, V3 a) { return mk(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b)
{
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double len(V3 a) { return sqrt(dot(a, a)); }
__device__ __forceinline__ V3 ld3(const double *p, int64_t i) { return mk(p[3 * i], p[3 * i + 1], p[3 * i + 2]); }

struct Tri {
    V3 a[3];
};
__device__ __forceinline__ Tri load_tri(const double *xyz, const int32_t *tri, int64_t c)
{
    Tri T;
    for (int i = 0; i < 3; ++i) T.a[i] = ld3(xyz, tri[3 * c + i]);
    return T;
}
__device__ __forceinline__ double area_of(const Tri &T) { return 0.5 * len(cross(T.a[1] - T.a[0], T.a[2] - T.a[0])); }
__device__ __forceinline__ V3 point(const Tri &T, double l0, double l1, double l2)
{
    return l0 * T.a[0] + l1 * T.a[1] + l2 * T.a[2];
}

// Moments of one source-triangle integral.
struct Mom {
    double I0;     // int 1/R
    V3 Iu;         // int (r' - p)/R
    double Sx[4];  // int x^p/R, x = R/dt - j (p = 3 with the x-moments only)
    V3 W;          // int (r - r')/R^3
    V3 Iux;        // int x (r' - p)/R          (x-moments: quadratic temporal bases)
    V3 Wx[2];      // int x^a (r - r')/R^3, a = 1, 2
};

__device__ __forceinline__ void mom_zero(Mom &m)
{
    m.I0 = 0.0;
    m.Iu = mk(0, 0, 0);
    m.Sx[0] = m.Sx[1] = m.Sx[2] = m.Sx[3] = 0.0;
    m.W = mk(0, 0, 0);
    m.Iux = mk(0, 0, 0);
    m.Wx[0] = m.Wx[1] = mk(0, 0, 0);
}

// Radial closed forms between R = lo and R = hi (lo >= |d|), rho =
// sqrt(R^2 - d^2): int dR, int rho dR, int x^a dR, d int dR/R^2, int rho/R^2 dR;
// with XM also int x rho dR, d int x^a/R^2 dR and int x^a rho/R^2 dR (a = 1,
// 2) from x = R/dt - j and the antiderivatives of rho R (rho^3/3) and rho/R
// (rho - |d| acos(|d|/R)).
template <bool WA, bool WS, bool WW, bool XM>
__device__ __forceinline__ void radial_add(double lo, double hi, double d, double d2, bool lo_plane,
                                           double jsh, double inv_dt, double dt, double wscal,
                                           V3 wvec, V3 nrm, bool coplanar, Mom &m)
{
    double slo = sqrt(fmax(lo * lo - d2, 0.0));
    double shi = sqrt(fmax(hi * hi - d2, 0.0));
    double P1 = 0.0;
    if (WA || (WW && XM)) {
        double lg = (d2 > 0.0 && lo + slo > 0.0) ? log((hi + shi) / (lo + slo)) : 0.0;
        P1 = 0.5 * (hi * shi - lo * slo) - 0.5 * d2 * lg;
    }
    if (WA) {
        m.I0 += wscal * (hi - lo);
        m.Iu = m.Iu + P1 * wvec;
        if (XM) {
            const double P1x = inv_dt * (shi * shi * shi - slo * slo * slo) * (1.0 / 3.0) - jsh * P1;
            m.Iux = m.Iux + P1x * wvec;
        }
    }
    if (WS) {
        double xl = lo * inv_dt - jsh, xh = hi * inv_dt - jsh;
        m.Sx[0] += wscal * dt * (xh - xl);
        m.Sx[1] += wscal * dt * (xh * xh - xl * xl) * 0.5;
        m.Sx[2] += wscal * dt * (xh * xh * xh - xl * xl * xl) * (1.0 / 3.0);
        if (XM) m.Sx[3] += wscal * dt * (xh * xh * xh * xh - xl * xl * xl * xl) * 0.25;
    }
    if (WW && !coplanar) {
        double dQ0, Q1;
        if (lo_plane) {
            dQ0 = (d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0)) - d / hi;
            Q1 = -shi / hi + log(hi + shi) - (lo > 0.0 ? log(lo) : 0.0);
        } else {
            dQ0 = d / lo - d / hi;
            Q1 = -shi / hi + slo / lo + log((hi + shi) / (lo + slo));
        }
        m.W = m.W + (wscal * dQ0) * nrm - Q1 * wvec;
        if (XM) {
            const double ad = fabs(d);
            const double flog = lo > 0.0 ? log(hi / lo) : 0.0;
            const double acl = lo > 0.0 ? acos(fmin(1.0, ad / lo)) : 0.0, ach = acos(fmin(1.0, ad / hi));
            const double G1 = (shi - ad * ach) - (slo - ad * acl);
            const double dQx1 = d * inv_dt * flog - jsh * dQ0, Qx1 = inv_dt * G1 - jsh * Q1;
            const double dQx2 = d * inv_dt * inv_dt * (hi - lo) - 2.0 * jsh * d * inv_dt * flog + jsh * jsh * dQ0;
            const double Qx2 = inv_dt * inv_dt * P1 - 2.0 * jsh * inv_dt * G1 + jsh * jsh * Q1;
            m.Wx[0] = m.Wx[0] + (wscal * dQx1) * nrm - Qx1 * wvec;
            m.Wx[1] = m.Wx[1] + (wscal * dQx2) * nrm - Qx2 * wvec;
        }
    }
}

// Integral over source triangle T from test point r on s_lo < R <= s_hi
// (XM: also the x-moments of the quadratic temporal bases).
template <bool WA, bool WS, bool WW, bool XM = false>
__device__ void inner(const Tri &T, V3 r, double s_lo, double s_hi, double jsh, double dt, int ng,
                      double coplanar_tol, Mom &m)
{
    mom_zero(m);
    V3 e1 = T.a[1] - T.a[0], e2 = T.a[2] - T.a[0];
    V3 nrm = cross(e1, e2);
    nrm = (1.0 / len(nrm)) * nrm;
    double d = dot(r - T.a[0], nrm);
    double ad = fabs(d), d2 = d * d;
    V3 p = r - d * nrm;
    bool coplanar = ad <= coplanar_tol * fmax(len(e1), len(e2));
    double R_lo = fmax(s_lo, ad);
    bool lo_plane = !(s_lo > ad);
    if (!(s_hi > R_lo)) return;
    const double inv_dt = 1.0 / dt;
    const bool finite_hi = !isinf(s_hi);
    for (int i = 0; i < 3; ++i) {
        V3 a = T.a[i], b = T.a[(i + 1) % 3];
        V3 et = b - a;
        double L = len(et);
        et = (1.0 / L) * et;
        V3 ap = a - p;
        double ta = dot(ap, et), tb = ta + L;
        V3 wh = ap - ta * et;
        double h = len(wh);
        if (h <= 1e-12 * L) continue;
        V3 eh = (1.0 / h) * wh;
        double sig = dot(cross(eh, et), nrm) > 0.0 ? 1.0 : -1.0;
        double sa = asinh(ta / h), sb = asinh(tb / h);
        double brk[6];
        int nb = 0;
        brk[nb++] = sa;
        double hd2 = h * h + d2;
        if (s_lo * s_lo > hd2) {
            double ps = asinh(sqrt(s_lo * s_lo - hd2) / h);
            if (-ps > sa && -ps < sb) brk[nb++] = -ps;
            if (ps > sa && ps < sb) brk[nb++] = ps;
        }
        if (finite_hi && s_hi * s_hi > hd2) {
            double ps = asinh(sqrt(s_hi * s_hi - hd2) / h);
            if (-ps > sa && -ps < sb) brk[nb++] = -ps;
            if (ps > sa && ps < sb) brk[nb++] = ps;
        }
        brk[nb++] = sb;
        for (int u = 1; u < nb; ++u) {  // insertion sort (<= 6 entries)
            double v = brk[u];
            int k = u - 1;
            while (k >= 0 && brk[k] > v) { brk[k + 1] = brk[k]; --k; }
            brk[k + 1] = v;
        }
        for (int s = 0; s + 1 < nb; ++s) {
            double lo = brk[s], hi = brk[s + 1];
            if (!(hi > lo)) continue;
            double mid = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
            double cm = cosh(mid);
            double Rm = sqrt(h * h * cm * cm + d2);
            if (!(Rm > R_lo)) continue;
            if (finite_hi && Rm >= s_hi) {
                double dpsi = atan(sinh(hi)) - atan(sinh(lo));
                double cu = tanh(hi) - tanh(lo);
                double su = 1.0 / cosh(hi) - 1.0 / cosh(lo);
                V3 du = cu * eh - su * et;
                Mom tmp;
                mom_zero(tmp);
                // constant radial pieces times the exact angular integrals
                radial_add<WA, WS, WW, XM>(R_lo, s_hi, d, d2, lo_plane, jsh, inv_dt, dt, sig * dpsi,
                                           sig * du, nrm, coplanar, tmp);
                m.I0 += tmp.I0;
                m.Iu = m.Iu + tmp.Iu;
                for (int k = 0; k < 4; ++k) m.Sx[k] += tmp.Sx[k];
                m.W = m.W + tmp.W;
                m.Iux = m.Iux + tmp.Iux;
                m.Wx[0] = m.Wx[0] + tmp.Wx[0];
                m.Wx[1] = m.Wx[1] + tmp.Wx[1];
                continue;
            }
            for (int g = 0; g < ng; ++g) {
                double sv = mid + half * c_gx[g];
                double ch = cosh(sv), sh = sinh(sv);
                double Rhi = sqrt(h * h * ch * ch + d2);
                double wgt = sig * half * c_gw[g] / ch;
                V3 u = (1.0 / ch) * (eh + sh * et);
                radial_add<WA, WS, WW, XM>(R_lo, Rhi, d, d2, lo_plane, jsh, inv_dt, dt, wgt, wgt * u, nrm,
                                           coplanar, m);
            }
        }
    }
}

// smallest / largest distance from r to triangle T
__device__ void dist_range(const Tri &T, V3 r, double &dmin, double &dmax)
{
    dmax = fmax(fmax(len(T.a[0] - r), len(T.a[1] - r)), len(T.a[2] - r));
    V3 n = cross(T.a[1] - T.a[0], T.a[2] - T.a[0]);
    n = (1.0 / len(n)) * n;
    double d = dot(r - T.a[0], n);
    V3 q = r - d * n;
    bool inside = true;
    for (int i = 0; i < 3; ++i) {
        V3 a = T.a[i], b = T.a[(i + 1) % 3];
        if (dot(cross(b - a, q - a), n) < 0.0) inside = false;
    }
    if (inside) {
        dmin = fabs(d);
        return;
    }
    double best = 1e300;
    for (int i = 0; i < 3; ++i) {
        V3 a = T.a[i], b = T.a[(i + 1) % 3];
        V3 ab = b - a;
        double t = dot(r - a, ab) / dot(ab, ab);
        t = fmin(1.0, fmax(0.0, t));
        best = fmin(best, len(r - (a + t * ab)));
    }
    dmin = best;
}

__device__ __forceinline__ bool share_vertex(const int32_t *tri, int64_t c1, int64_t c2)
{
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k)
            if (tri[3 * c1 + i] == tri[3 * c2 + k]) return true;
    return false;
}

// RT0 field with outward fluxes F on triangle T (area A) at r
__device__ __forceinline__ V3 rt0(const Tri &T, double A, const double *F, V3 r)
{
    double s = 0.5 / A;
    return (s * F[0]) * (r - T.a[0]) + (s * F[1]) * (r - T.a[1]) + (s * F[2]) * (r - T.a[2]);
}

// ------------------------------------------------------------------ Gram
__global__ void k_gram(AsmArgs g, double *G)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.nf) return;
    int64_t c = g.fparent[t];
    Tri P = load_tri(g.fxyz, g.ftri, t);
    Tri Q = load_tri(g.xyz, g.tri, c);
    double A = area_of(P), Ac = area_of(Q);
    V3 n = cross(Q.a[1] - Q.a[0], Q.a[2] - Q.a[0]);
    n = (1.0 / len(n)) * n;
    for (int e = g.bc_off[t]; e < g.bc_off[t + 1]; ++e) {
        const double *F = g.bc_flux + 3 * e;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < 3; ++q) {
            double l0, l1, l2, w;
            tri3_point(q, l0, l1, l2, w);
            V3 r = point(P, l0, l1, l2);
            V3 ng = cross(n, rt0(P, A, F, r));
            for (int b = 0; b < 3; ++b) {
                V3 f = (g.tri_sign[3 * c + b] / (2.0 * Ac)) * (r - Q.a[b]);
                acc[b] += w * A * dot(ng, f);
            }
        }
        int64_t m = g.bc_edge[e];
        for (int b = 0; b < 3; ++b) atomicAdd(&G[m * g.ne + g.tri_edge[3 * c + b]], acc[b]);
    }
}

// --------------------------------------------------- retarded, coarse x coarse
// thread per (test c, source cs); shells [j0, j1]; temporal bases of order
// OR (1: hat functions, 2: quadratic): V[(j-j0)][a][m][n] (x^a, a < OR),
// S[(j-j0)][p][c][cs] (x^p/(4 pi R), p < OR + 2).
template <int OR>
__global__ __launch_bounds__(128) void k_ret_coarse(AsmArgs g, int64_t j0, int64_t j1, double *V, double *S)
{
    constexpr int VP = OR, SP = OR + 2;
    constexpr bool XM = OR > 1;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.nc * g.nc) return;
    int64_t c = idx / g.nc, cs = idx % g.nc;
    Tri P = load_tri(g.xyz, g.tri, c);
    Tri Q = load_tri(g.xyz, g.tri, cs);
    double A = area_of(P), As = area_of(Q);
    // shell range of the pair (bounding spheres about the centroids)
    V3 gc = (1.0 / 3.0) * (P.a[0] + P.a[1] + P.a[2]), gs = (1.0 / 3.0) * (Q.a[0] + Q.a[1] + Q.a[2]);
    double rc = fmax(fmax(len(P.a[0] - gc), len(P.a[1] - gc)), len(P.a[2] - gc));
    double rs = fmax(fmax(len(Q.a[0] - gs), len(Q.a[1] - gs)), len(Q.a[2] - gs));
    double dc = len(gc - gs);
    int64_t jlo = (int64_t)floor(fmax(dc - rc - rs, 0.0) / g.dt) - 1;
    int64_t jhi = (int64_t)floor((dc + rc + rs) / g.dt);
    jlo = jlo < j0 ? j0 : jlo;
    jhi = jhi > j1 ? j1 : jhi;
    if (jlo > jhi) return;
    const int64_t nsh = j1 - j0 + 1;
    V3 nq = cross(Q.a[1] - Q.a[0], Q.a[2] - Q.a[0]);
    nq = (1.0 / len(nq)) * nq;
    int32_t me[3], ms[3], ne_[3], ns_[3];
    for (int a = 0; a < 3; ++a) {
        me[a] = g.tri_edge[3 * c + a];
        ms[a] = g.tri_sign[3 * c + a];
        ne_[a] = g.tri_edge[3 * cs + a];
        ns_[a] = g.tri_sign[3 * cs + a];
    }
    for (int64_t j = jlo; j <= jhi; ++j) {
        double vacc[VP][3][3];
        double sacc[SP];
        for (int x = 0; x < VP; ++x)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) vacc[x][a][b] = 0.0;
        for (int p = 0; p < SP; ++p) sacc[p] = 0.0;
        bool any = false;
        for (int q = 0; q < 7; ++q) {
            double l0, l1, l2, w;
            radon7_point(q, l0, l1, l2, w);
            V3 r = point(P, l0, l1, l2);
            double dmin, dmax;
            dist_range(Q, r, dmin, dmax);
            int64_t qlo = (int64_t)floor(dmin / g.dt) - 1, qhi = (int64_t)floor(dmax / g.dt);
            if (j < qlo || j > qhi) continue;
            Mom mo;
            inner<true, true, false, XM>(Q, r, j * g.dt, (j + 1) * g.dt, (double)j, g.dt, g.ng, 1e-12, mo);
            any = true;
            double wq = w * A;
            for (int p = 0; p < SP; ++p) sacc[p] += wq * mo.Sx[p];
            V3 pp = r - dot(r - Q.a[0], nq) * nq;
            for (int b = 0; b < 3; ++b) {
                double sb = wq * ns_[b] / (2.0 * As);
                for (int x = 0; x < VP; ++x) {
                    // x^0: int (r' - p)/R + (p - Q_b) int 1/R; x^1: the same with x-weights
                    V3 vb = x == 0 ? mo.Iu + mo.I0 * (pp - Q.a[b]) : mo.Iux + mo.Sx[1] * (pp - Q.a[b]);
                    for (int a = 0; a < 3; ++a) {
                        V3 fa = (ms[a] / (2.0 * A)) * (r - P.a[a]);
                        vacc[x][a][b] += sb * dot(fa, vb);
                    }
                }
            }
        }
        if (!any) continue;
        int64_t jj = j - j0;
        for (int p = 0; p < SP; ++p) S[((jj * SP + p) * g.nc + c) * g.nc + cs] = sacc[p] / kFourPi;
        for (int x = 0; x < VP; ++x)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    atomicAdd(&V[((jj * VP + x) * g.ne + me[a]) * g.ne + ne_[b]], vacc[x][a][b] / kFourPi);
    }
    (void)nsh;
}

// ---------------------------------------------- retarded, BC x RWG (MFIE K)
// thread per (coarse vertex v: test dual cell, source triangle cs);
// N[(j-j0)][a][m][n] (x^a, a <= OR)
template <int OR>
__global__ __launch_bounds__(128) void k_ret_bc(AsmArgs g, int64_t j0, int64_t j1, double *N)
{
    constexpr int NP = OR + 1;
    constexpr bool XM = OR > 1;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.nv * g.nc) return;
    int64_t v = idx / g.nc, cs = idx % g.nc;
    Tri Q = load_tri(g.xyz, g.tri, cs);
    double As = area_of(Q);
    // distance range from the dual cell (ball about v of radius = farthest fine vertex)
    V3 pv = ld3(g.xyz, v);
    double rv = 0.0;
    for (int k = g.vcell_off[v]; k < g.vcell_off[v + 1]; ++k) {
        int64_t t = g.vcell_tri[k];
        for (int i = 0; i < 3; ++i) rv = fmax(rv, len(ld3(g.fxyz, g.ftri[3 * t + i]) - pv));
    }
    V3 gs = (1.0 / 3.0) * (Q.a[0] + Q.a[1] + Q.a[2]);
    double rs = fmax(fmax(len(Q.a[0] - gs), len(Q.a[1] - gs)), len(Q.a[2] - gs));
    double dc = len(pv - gs);
    int64_t jlo = (int64_t)floor(fmax(dc - rv - rs, 0.0) / g.dt) - 1;
    int64_t jhi = (int64_t)floor((dc + rv + rs) / g.dt);
    jlo = jlo < j0 ? j0 : jlo;
    jhi = jhi > j1 ? j1 : jhi;
    if (jlo > jhi) return;
    const int nval = g.vedge_off[v + 1] - g.vedge_off[v];
    int32_t nb_[3], sb_[3];
    for (int b = 0; b < 3; ++b) {
        nb_[b] = g.tri_edge[3 * cs + b];
        sb_[b] = g.tri_sign[3 * cs + b];
    }
    for (int64_t j = jlo; j <= jhi; ++j) {
        double acc[NP][kMaxValence][3];
        for (int x = 0; x < NP; ++x)
            for (int i = 0; i < kMaxValence; ++i) acc[x][i][0] = acc[x][i][1] = acc[x][i][2] = 0.0;
        bool any = false;
        for (int k = g.vcell_off[v]; k < g.vcell_off[v + 1]; ++k) {
            int64_t t = g.vcell_tri[k];
            if (g.fparent[t] == cs) continue;  // coplanar: integrand is zero
            Tri P = load_tri(g.fxyz, g.ftri, t);
            double A = area_of(P);
            for (int q = 0; q < 3; ++q) {
                double l0, l1, l2, w;
                tri3_point(q, l0, l1, l2, w);
                V3 r = point(P, l0, l1, l2);
                double dmin, dmax;
                dist_range(Q, r, dmin, dmax);
                int64_t qlo = (int64_t)floor(dmin / g.dt) - 1, qhi = (int64_t)floor(dmax / g.dt);
                if (j < qlo || j > qhi) continue;
                Mom mo;
                inner<false, false, true, XM>(Q, r, j * g.dt, (j + 1) * g.dt, (double)j, g.dt, g.ng,
                                              g.coplanar_tol, mo);
                any = true;
                double wq = w * A;
                for (int x = 0; x < NP; ++x) {
                    const V3 W = x == 0 ? mo.W : mo.Wx[x - 1];
                    V3 wx[3];
                    for (int b = 0; b < 3; ++b) wx[b] = (wq * sb_[b] / (2.0 * As)) * cross(W, r - Q.a[b]);
                    for (int e = g.bc_off[t]; e < g.bc_off[t + 1]; ++e) {
                        V3 gv = rt0(P, A, g.bc_flux + 3 * e, r);
                        int li = g.bc_local[e];
                        for (int b = 0; b < 3; ++b) acc[x][li][b] += dot(wx[b], gv);
                    }
                }
            }
        }
        if (!any) continue;
        int64_t jj = j - j0;
        for (int x = 0; x < NP; ++x)
            for (int i = 0; i < nval; ++i) {
                int64_t m = g.vedge[g.vedge_off[v] + i];
                for (int b = 0; b < 3; ++b)
                    atomicAdd(&N[((jj * NP + x) * g.ne + m) * g.ne + nb_[b]], acc[x][i][b] / kFourPi);
            }
    }
}

// ------------------------------------------------------- Yukawa, BC x BC
// thread per (coarse vertex v: test dual cell, fine source triangle ts).
// Zs[m][n] += int int g_m . g_n e^{-kR}/(4 pi R);
// D[v][owner(ts)] += sum int int e^{-kR}/(4 pi R) / (A_t A_ts).
__global__ __launch_bounds__(128) void k_yuk_bcbc(AsmArgs g, double kappa, double *Zs, double *D)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.nv * g.nf) return;
    int64_t v = idx / g.nf, ts = idx % g.nf;
    Tri Q = load_tri(g.fxyz, g.ftri, ts);
    double As = area_of(Q);
    V3 nq = cross(Q.a[1] - Q.a[0], Q.a[2] - Q.a[0]);
    nq = (1.0 / len(nq)) * nq;
    const int nval = g.vedge_off[v + 1] - g.vedge_off[v];
    double Y[kMaxValence][3];
    for (int i = 0; i < kMaxValence; ++i) Y[i][0] = Y[i][1] = Y[i][2] = 0.0;
    double J = 0.0;
    int64_t ps = g.fparent[ts];
    for (int k = g.vcell_off[v]; k < g.vcell_off[v + 1]; ++k) {
        int64_t t = g.vcell_tri[k];
        Tri P = load_tri(g.fxyz, g.ftri, t);
        double A = area_of(P);
        bool near = share_vertex(g.tri, g.fparent[t], ps);
        double Jt = 0.0;
        for (int q = 0; q < 3; ++q) {
            double l0, l1, l2, w;
            tri3_point(q, l0, l1, l2, w);
            V3 r = point(P, l0, l1, l2);
            double I = 0.0;
            V3 Vb[3] = {mk(0, 0, 0), mk(0, 0, 0), mk(0, 0, 0)};
            if (near) {
                Mom mo;
                inner<true, false, false>(Q, r, 0.0, INFINITY, 0.0, 1.0, g.ng, 1e-12, mo);
                V3 pp = r - dot(r - Q.a[0], nq) * nq;
                I += mo.I0 / kFourPi;
                for (int b = 0; b < 3; ++b) Vb[b] = Vb[b] + (1.0 / kFourPi) * (mo.Iu + mo.I0 * (pp - Q.a[b]));
            }
            for (int s = 0; s < 7; ++s) {
                double m0, m1, m2, ws;
                radon7_point(s, m0, m1, m2, ws);
                V3 rs = point(Q, m0, m1, m2);
                double R = len(r - rs);
                double x = kappa * R;
                double G;
                if (near) G = (x == 0.0) ? -kappa / kFourPi : expm1(-x) / (R * kFourPi);
                else G = exp(-x) / (kFourPi * R);
                double wsG = ws * As * G;
                I += wsG;
                for (int b = 0; b < 3; ++b) Vb[b] = Vb[b] + wsG * (rs - Q.a[b]);
            }
            double wq = w * A;
            Jt += wq * I;
            double sc = wq / (4.0 * A * As);
            for (int e = g.bc_off[t]; e < g.bc_off[t + 1]; ++e) {
                const double *F = g.bc_flux + 3 * e;
                int li = g.bc_local[e];
                for (int b = 0; b < 3; ++b) {
                    double s = 0.0;
                    for (int a = 0; a < 3; ++a) s += F[a] * dot(r - P.a[a], Vb[b]);
                    Y[li][b] += sc * s;
                }
            }
        }
        J += Jt / (A * As);
    }
    for (int es = g.bc_off[ts]; es < g.bc_off[ts + 1]; ++es) {
        const double *F = g.bc_flux + 3 * es;
        int64_t n = g.bc_edge[es];
        for (int i = 0; i < nval; ++i) {
            int64_t m = g.vedge[g.vedge_off[v] + i];
            atomicAdd(&Zs[m * g.ne + n], Y[i][0] * F[0] + Y[i][1] * F[1] + Y[i][2] * F[2]);
        }
    }
    atomicAdd(&D[v * g.nv + g.fowner[ts]], J);
}

// ((1 + x) e^{-x} - 1) / x^2
__device__ __forceinline__ double mf_phi(double x)
{
    if (x < 0.1) {
        const double c[8] = {-1.0 / 2.0, 1.0 / 3.0, -1.0 / 8.0, 1.0 / 30.0, -1.0 / 144.0, 1.0 / 840.0,
                             -1.0 / 5760.0, 1.0 / 45360.0};
        double s = c[7];
        for (int i = 6; i >= 0; --i) s = s * x + c[i];
        return s;
    }
    return ((1.0 + x) * exp(-x) - 1.0) / (x * x);
}

// ------------------------------------------------------- Yukawa MFIE, BC x RWG
// thread per (coarse vertex v: test dual cell, coarse source cs)
__global__ __launch_bounds__(128) void k_yuk_mfie(AsmArgs g, double kappa, double *M)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.nv * g.nc) return;
    int64_t v = idx / g.nc, cs = idx % g.nc;
    Tri Q = load_tri(g.xyz, g.tri, cs);
    double As = area_of(Q);
    const int nval = g.vedge_off[v + 1] - g.vedge_off[v];
    int32_t nb_[3], sb_[3];
    for (int b = 0; b < 3; ++b) {
        nb_[b] = g.tri_edge[3 * cs + b];
        sb_[b] = g.tri_sign[3 * cs + b];
    }
    double acc[kMaxValence][3];
    for (int i = 0; i < kMaxValence; ++i) acc[i][0] = acc[i][1] = acc[i][2] = 0.0;
    for (int k = g.vcell_off[v]; k < g.vcell_off[v + 1]; ++k) {
        int64_t t = g.vcell_tri[k];
        if (g.fparent[t] == cs) continue;
        Tri P = load_tri(g.fxyz, g.ftri, t);
        double A = area_of(P);
        bool near = share_vertex(g.tri, g.fparent[t], cs);
        for (int q = 0; q < 3; ++q) {
            double l0, l1, l2, w;
            tri3_point(q, l0, l1, l2, w);
            V3 r = point(P, l0, l1, l2);
            V3 W = mk(0, 0, 0);
            if (near) {
                Mom mo;
                inner<false, false, true>(Q, r, 0.0, INFINITY, 0.0, 1.0, g.ng, g.coplanar_tol, mo);
                W = (1.0 / kFourPi) * mo.W;
            }
            for (int s = 0; s < 7; ++s) {
                double m0, m1, m2, ws;
                radon7_point(s, m0, m1, m2, ws);
                V3 rs = point(Q, m0, m1, m2);
                V3 dr = r - rs;
                double R = len(dr);
                double x = kappa * R;
                double K = near ? kappa * kappa * mf_phi(x) / R : (1.0 + x) * exp(-x) / (R * R * R);
                W = W + (ws * As * K / kFourPi) * dr;
            }
            double wq = w * A;
            V3 wx[3];
            for (int b = 0; b < 3; ++b) wx[b] = (wq * sb_[b] / (2.0 * As)) * cross(W, r - Q.a[b]);
            for (int e = g.bc_off[t]; e < g.bc_off[t + 1]; ++e) {
                V3 gv = rt0(P, A, g.bc_flux + 3 * e, r);
                int li = g.bc_local[e];
                for (int b = 0; b < 3; ++b) acc[li][b] += dot(wx[b], gv);
            }
        }
    }
    for (int i = 0; i < nval; ++i) {
        int64_t m = g.vedge[g.vedge_off[v] + i];
        for (int b = 0; b < 3; ++b) atomicAdd(&M[m * g.ne + nb_[b]], acc[i][b]);
    }
}

// --------------------------------------------------------------- gathers
// Laplacians: L_Sigma = Sigma^T Sigma (+ 1/n everywhere), L_Lambda likewise
__global__ void k_lap_sigma(AsmArgs g, double *L)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nc) return;
    double inv = 1.0 / (double)g.nc;
    for (int64_t k = 0; k < g.nc; ++k) L[c * g.nc + k] = inv;
    L[c * g.nc + c] += 3.0;
    for (int a = 0; a < 3; ++a) {
        int64_t e = g.tri_edge[3 * c + a];
        int64_t o = g.cells[2 * e] == c ? g.cells[2 * e + 1] : g.cells[2 * e];
        L[c * g.nc + o] -= 1.0;
    }
}
__global__ void k_lap_lambda(AsmArgs g, double *L)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.nv) return;
    double inv = 1.0 / (double)g.nv;
    for (int64_t k = 0; k < g.nv; ++k) L[v * g.nv + k] = inv;
    for (int q = g.vedge_off[v]; q < g.vedge_off[v + 1]; ++q) {
        int64_t e = g.vedge[q];
        int64_t o = g.edges[2 * e] == v ? g.edges[2 * e + 1] : g.edges[2 * e];
        L[v * g.nv + v] += 1.0;
        L[v * g.nv + o] -= 1.0;
    }
}
// out -= 1/n everywhere (turns (L + 11^T/n)^{-1} into the pseudo-inverse)
__global__ void k_sub_const(int64_t n, double *X)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n * n) X[i] -= 1.0 / (double)n;
}
// P[m][n] = sum_{a in {i0(m), i1(m)}, b in {i0(n), i1(n)}} s_a s_b Lp[a][b],
// with (i0, i1) = (first, second) incidence and signs (+1, -1)
__global__ void k_proj(int64_t ne, const int32_t *pairs, int sign_first, const double *Lp, int64_t nl, double *P)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ne * ne) return;
    int64_t m = idx / ne, n = idx % ne;
    int64_t a0 = pairs[2 * m], a1 = pairs[2 * m + 1], b0 = pairs[2 * n], b1 = pairs[2 * n + 1];
    double v = Lp[a0 * nl + b0] - Lp[a0 * nl + b1] - Lp[a1 * nl + b0] + Lp[a1 * nl + b1];
    P[idx] = v;
    (void)sign_first;
}
// Z^h[m][n] = -(1/kappa) sum Lam_ma Lam_nb D[a][b] / (4 N_a N_b)
__global__ void k_zh(AsmArgs g, double kappa, const double *D, double *Zh)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.ne * g.ne) return;
    int64_t m = idx / g.ne, n = idx % g.ne;
    int64_t am[2] = {g.edges[2 * m + 1], g.edges[2 * m]}, an[2] = {g.edges[2 * n + 1], g.edges[2 * n]};
    double sg[2] = {1.0, -1.0};
    double s = 0.0;
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 2; ++k)
            s += sg[i] * sg[k] * D[am[i] * g.nv + an[k]] /
                 (4.0 * (double)g.valence[am[i]] * (double)g.valence[an[k]]);
    Zh[idx] = -s / kappa;
}
// B_k[m][n] = -T0 sum Sig_ma Sig_nb Sq[a][b] / (A_a A_b), Sq from shell moments
__global__ void k_bk(AsmArgs g, const double *Sk, const double *Sk1, const double *Sk2, double T0, double *B)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.ne * g.ne) return;
    int64_t m = idx / g.ne, n = idx % g.ne;
    int64_t am[2] = {g.cells[2 * m], g.cells[2 * m + 1]}, an[2] = {g.cells[2 * n], g.cells[2 * n + 1]};
    double sg[2] = {1.0, -1.0};
    const int64_t nc2 = g.nc * g.nc;
    double s = 0.0;
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 2; ++k) {
            int64_t o = am[i] * g.nc + an[k];
            // q_0 on shells k, k-1, k-2 (x = R/dt - j): (1-x)^2/2, 1/2 + x - x^2, x^2/2
            double sq = 0.0;
            if (Sk) sq += 0.5 * (Sk[o] - 2.0 * Sk[nc2 + o] + Sk[2 * nc2 + o]);
            if (Sk1) sq += 0.5 * Sk1[o] + Sk1[nc2 + o] - Sk1[2 * nc2 + o];
            if (Sk2) sq += 0.5 * Sk2[2 * nc2 + o];
            s += sg[i] * sg[k] * sq / (g.area[am[i]] * g.area[an[k]]);
        }
    B[idx] = -T0 * s;
}
// Sq_k[a][b] = q_0 of lag k on the shell moments of triangles a, b (shells
// k, k-1, k-2; x = R/dt - j): (1-x)^2/2, 1/2 + x - x^2, x^2/2
__global__ void k_sq(int64_t nc, const double *Sk, const double *Sk1, const double *Sk2, double *Sq)
{
    int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nc2 = nc * nc;
    if (o >= nc2) return;
    double sq = 0.0;
    if (Sk) sq += 0.5 * (Sk[o] - 2.0 * Sk[nc2 + o] + Sk[2 * nc2 + o]);
    if (Sk1) sq += 0.5 * Sk1[o] + Sk1[nc2 + o] - Sk1[2 * nc2 + o];
    if (Sk2) sq += 0.5 * Sk2[2 * nc2 + o];
    Sq[o] = sq;
}
// symmetrise the coarse shell moments S [np][nc][nc] in place
__global__ void k_sym_s(int64_t nc, int np, double *S)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nc * nc) return;
    int64_t i = idx / nc, j = idx % nc;
    if (j <= i) return;
    for (int p = 0; p < np; ++p) {
        double *X = S + p * nc * nc;
        double v = 0.5 * (X[i * nc + j] + X[j * nc + i]);
        X[i * nc + j] = v;
        X[j * nc + i] = v;
    }
}
// A_k = -(V_k - V_{k-1})/dt ; C_k = (k+1) N_k + (1-k) N_{k-1} (+ G/2 at k = 0)
__global__ void k_lag_ac(int64_t nn, int64_t k, double dt, const double *Vk, const double *Vk1,
                         const double *Nk, const double *Nk1, const double *G, double *A, double *C)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    double vk = Vk ? Vk[i] : 0.0, vk1 = Vk1 ? Vk1[i] : 0.0;
    double nk = Nk ? Nk[i] : 0.0, nk1 = Nk1 ? Nk1[i] : 0.0;
    A[i] = -(vk - vk1) / dt;
    double c = (k + 1.0) * nk + (1.0 - k) * nk1;
    if (k == 0) c += 0.5 * G[i];
    C[i] = c;
}
// out = base_c * base + sum_t c[t] * p[t] (elementwise; null terms skipped):
// the lag combinations of temporal bases of higher order
__global__ void k_lincomb(int64_t n, LinTerms t, double base_c, const double *base, double *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = base ? base_c * base[i] : 0.0;
    for (int q = 0; q < t.n; ++q)
        if (t.p[q]) v += t.c[q] * t.p[q][i];
    out[i] = v;
}
// B_k[m][n] = -T0 sum Sig_ma Sig_nb Sq[a][b] / (A_a A_b) from a formed Sq_k
__global__ void k_bk_sq(AsmArgs g, const double *Sq, double T0, double *B)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.ne * g.ne) return;
    int64_t m = idx / g.ne, n = idx % g.ne;
    int64_t am[2] = {g.cells[2 * m], g.cells[2 * m + 1]}, an[2] = {g.cells[2 * n], g.cells[2 * n + 1]};
    double sg[2] = {1.0, -1.0};
    double s = 0.0;
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 2; ++k)
            s += sg[i] * sg[k] * Sq[am[i] * g.nc + an[k]] / (g.area[am[i]] * g.area[an[k]]);
    B[idx] = -T0 * s;
}

// X = alpha X + beta Y + gamma Z (elementwise)
__global__ void k_lin3(int64_t n, double *X, double a, const double *Y, double b, const double *Z, double c)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = a * X[i];
    if (Y) v += b * Y[i];
    if (Z) v += c * Z[i];
    X[i] = v;
}

static unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_sq(hipStream_t s, int64_t nc, const double *Sk, const double *Sk1, const double *Sk2, double *Sq)
{
    hipLaunchKernelGGL(k_sq, dim3(nblk(nc * nc, 256)), dim3(256), 0, s, nc, Sk, Sk1, Sk2, Sq);
}
void launch_gram(hipStream_t s, const AsmArgs &g, double *G)
{
    hipLaunchKernelGGL(k_gram, dim3(nblk(g.nf, 128)), dim3(128), 0, s, g, G);
}
void launch_ret_coarse(hipStream_t s, const AsmArgs &g, int order, int64_t j0, int64_t j1, double *V, double *S)
{
    if (order == 2)
        hipLaunchKernelGGL(k_ret_coarse<2>, dim3(nblk(g.nc * g.nc, 128)), dim3(128), 0, s, g, j0, j1, V, S);
    else
        hipLaunchKernelGGL(k_ret_coarse<1>, dim3(nblk(g.nc * g.nc, 128)), dim3(128), 0, s, g, j0, j1, V, S);
}
void launch_ret_bc(hipStream_t s, const AsmArgs &g, int order, int64_t j0, int64_t j1, double *N)
{
    if (order == 2)
        hipLaunchKernelGGL(k_ret_bc<2>, dim3(nblk(g.nv * g.nc, 128)), dim3(128), 0, s, g, j0, j1, N);
    else
        hipLaunchKernelGGL(k_ret_bc<1>, dim3(nblk(g.nv * g.nc, 128)), dim3(128), 0, s, g, j0, j1, N);
}
void launch_yuk_bcbc(hipStream_t s, const AsmArgs &g, double kappa, double *Zs, double *D)
{
    hipLaunchKernelGGL(k_yuk_bcbc, dim3(nblk(g.nv * g.nf, 128)), dim3(128), 0, s, g, kappa, Zs, D);
}
void launch_yuk_mfie(hipStream_t s, const AsmArgs &g, double kappa, double *M)
{
    hipLaunchKernelGGL(k_yuk_mfie, dim3(nblk(g.nv * g.nc, 128)), dim3(128), 0, s, g, kappa, M);
}
void launch_laplacians(hipStream_t s, const AsmArgs &g, double *LS, double *LL)
{
    hipLaunchKernelGGL(k_lap_sigma, dim3(nblk(g.nc, 128)), dim3(128), 0, s, g, LS);
    hipLaunchKernelGGL(k_lap_lambda, dim3(nblk(g.nv, 128)), dim3(128), 0, s, g, LL);
}
void launch_sub_const(hipStream_t s, int64_t n, double *X)
{
    hipLaunchKernelGGL(k_sub_const, dim3(nblk(n * n, 256)), dim3(256), 0, s, n, X);
}
void launch_proj(hipStream_t s, int64_t ne, const int32_t *pairs, const double *Lp, int64_t nl, double *P)
{
    hipLaunchKernelGGL(k_proj, dim3(nblk(ne * ne, 256)), dim3(256), 0, s, ne, pairs, 1, Lp, nl, P);
}
void launch_zh(hipStream_t s, const AsmArgs &g, double kappa, const double *D, double *Zh)
{
    hipLaunchKernelGGL(k_zh, dim3(nblk(g.ne * g.ne, 256)), dim3(256), 0, s, g, kappa, D, Zh);
}
void launch_bk(hipStream_t s, const AsmArgs &g, const double *Sk, const double *Sk1, const double *Sk2,
               double T0, double *B)
{
    hipLaunchKernelGGL(k_bk, dim3(nblk(g.ne * g.ne, 256)), dim3(256), 0, s, g, Sk, Sk1, Sk2, T0, B);
}
void launch_sym_s(hipStream_t s, int64_t nc, int np, double *S)
{
    hipLaunchKernelGGL(k_sym_s, dim3(nblk(nc * nc, 256)), dim3(256), 0, s, nc, np, S);
}
void launch_lag_ac(hipStream_t s, int64_t nn, int64_t k, double dt, const double *Vk, const double *Vk1,
                   const double *Nk, const double *Nk1, const double *G, double *A, double *C)
{
    hipLaunchKernelGGL(k_lag_ac, dim3(nblk(nn, 256)), dim3(256), 0, s, nn, k, dt, Vk, Vk1, Nk, Nk1, G, A, C);
}
void launch_lincomb(hipStream_t s, int64_t n, const LinTerms &t, double base_c, const double *base, double *out)
{
    hipLaunchKernelGGL(k_lincomb, dim3(nblk(n, 256)), dim3(256), 0, s, n, t, base_c, base, out);
}
void launch_bk_sq(hipStream_t s, const AsmArgs &g, const double *Sq, double T0, double *B)
{
    hipLaunchKernelGGL(k_bk_sq, dim3(nblk(g.ne * g.ne, 256)), dim3(256), 0, s, g, Sq, T0, B);
}
void launch_lin3(hipStream_t s, int64_t n, double *X, double a, const double *Y, double b, const double *Z, double c)
{
    hipLaunchKernelGGL(k_lin3, dim3(nblk(n, 256)), dim3(256), 0, s, n, X, a, Y, b, Z, c);
}
void set_gauss(const double *x, const double *w, int n)
{
    (void)hipMemcpyToSymbol(HIP_SYMBOL(c_gx), x, sizeof(double) * n);
    (void)hipMemcpyToSymbol(HIP_SYMBOL(c_gw), w, sizeof(double) * n);
}

}  // namespace qhp
