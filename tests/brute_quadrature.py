"""Independent integrals of single matrix entries, to pin the oracle's
assembly (test infrastructure).

Nothing here comes from ``oracle/`` or the library except the mesh tables
(edge numbering, BC fluxes), which their own tests pin.  The basis functions
are built from their defining properties and the integrals from their
definitions (Sec. II-A, II-C, IV-A):

* a field of the lowest-order Raviart-Thomas space on a triangle,
  f(r) = alpha + beta (r - centroid) with alpha in the plane, is found by
  solving for the three outward edge fluxes it must have; the fluxes of the
  trial fields are integrated along the edges by Gauss-Legendre;
* the inner (source) integral over a triangle Q, restricted to the shell
  lo < R <= hi (R = |r - r'|), at one outer point r:
    - a = the point of Q closest to r; Q is the union of the fan triangles
      (a, q_i, q_i+1) of positive area, each parametrised by
      r' = a + u w(v), w(v) = q_i - a + v (q_i+1 - q_i), u, v in [0, 1]
      (Duffy), whose Jacobian 2 A_fan u cancels the 1/R singularity at a;
    - along each such ray R^2 = C - 2 B u + A u^2 grows with u (a is the
      closest point, so B <= 0), so the shell is exactly the u-interval
      between the roots of R = lo and R = hi; v is cut where a root reaches
      the far edge (u = 1);
    - Gauss-Legendre in u on pieces graded towards u = 0 on the length scale
      |r - a| / |w| (near-singular kernels), and in v on each piece;
* the outer (test) integral by the same symmetric rules the quadrature
  specification fixes (Radon's 7-point rule on coarse triangles, the 3-point
  rule on fine ones), written out here from the published values.
"""
from __future__ import annotations

import math

import numpy as np

FOUR_PI = 4.0 * math.pi

_GL = {}


def gl01(n):
    """Gauss-Legendre nodes and weights on [0, 1] (library routine)."""
    if n not in _GL:
        x, w = np.polynomial.legendre.leggauss(n)
        _GL[n] = (0.5 * (x + 1.0), 0.5 * w)
    return _GL[n]


def radon7_rule():
    """Radon's 7-point rule of degree 5 (barycentric points, weights summing to 1)."""
    s = math.sqrt(15.0)
    a1, b1 = (9.0 - 2.0 * s) / 21.0, (6.0 + s) / 21.0
    a2, b2 = (9.0 + 2.0 * s) / 21.0, (6.0 - s) / 21.0
    pts = [(1 / 3, 1 / 3, 1 / 3), (a1, b1, b1), (b1, a1, b1), (b1, b1, a1), (a2, b2, b2), (b2, a2, b2), (b2, b2, a2)]
    w = [9.0 / 40.0] + [(155.0 + s) / 1200.0] * 3 + [(155.0 - s) / 1200.0] * 3
    return np.array(pts), np.array(w)


def three_point_rule():
    """The 3-point rule of degree 2 with points (2/3, 1/6, 1/6)."""
    return (np.array([(2 / 3, 1 / 6, 1 / 6), (1 / 6, 2 / 3, 1 / 6), (1 / 6, 1 / 6, 2 / 3)]),
            np.full(3, 1.0 / 3.0))


def area(P):
    return 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))


def rule_points(P, rule):
    """Points and weights (times the area) of a barycentric rule on triangle P."""
    bary, w = rule
    return bary @ P, w * area(P)


def rt0(P, fluxes):
    """The field of the lowest-order Raviart-Thomas space on triangle P whose
    outward flux through the edge opposite P[i] is fluxes[i]; returned as a
    function of points [..., 3]."""
    P = np.asarray(P, dtype=np.float64)
    n = np.cross(P[1] - P[0], P[2] - P[0])
    n /= np.linalg.norm(n)
    e1 = (P[1] - P[0]) / np.linalg.norm(P[1] - P[0])
    e2 = np.cross(n, e1)
    cen = P.mean(axis=0)
    xg, wg = gl01(4)
    basis = [lambda r: np.broadcast_to(e1, np.shape(r)), lambda r: np.broadcast_to(e2, np.shape(r)),
             lambda r: r - cen]
    M = np.zeros((3, 3))
    for i in range(3):
        a, b = P[(i + 1) % 3], P[(i + 2) % 3]
        t = b - a
        nu = np.cross(t, n)  # in-plane normal of edge (a, b)
        if np.dot(nu, a - P[i]) < 0:  # pointing away from the opposite vertex: outward
            nu = -nu
        nu /= np.linalg.norm(nu)
        pts = a[None, :] + xg[:, None] * t[None, :]
        L = np.linalg.norm(t)
        for k, f in enumerate(basis):
            M[i, k] = L * np.sum(wg * (f(pts) @ nu))
    coef = np.linalg.solve(M, np.asarray(fluxes, dtype=np.float64))

    def field(r):
        r = np.asarray(r, dtype=np.float64)
        return coef[0] * e1 + coef[1] * e2 + coef[2] * (r - cen)

    return field


def closest_point(Q, r):
    """Point of triangle Q closest to r."""
    best, bd = None, np.inf
    n = np.cross(Q[1] - Q[0], Q[2] - Q[0])
    n /= np.linalg.norm(n)
    p = r - np.dot(r - Q[0], n) * n
    # barycentric coordinates of the projection
    T = np.array([Q[0] - Q[2], Q[1] - Q[2]]).T
    lam = np.linalg.lstsq(T, p - Q[2], rcond=None)[0]
    l3 = 1.0 - lam.sum()
    if lam[0] >= 0 and lam[1] >= 0 and l3 >= 0:
        return p
    for i in range(3):
        a, b = Q[i], Q[(i + 1) % 3]
        t = np.clip(np.dot(r - a, b - a) / np.dot(b - a, b - a), 0.0, 1.0)
        c = a + t * (b - a)
        d = np.linalg.norm(r - c)
        if d < bd:
            best, bd = c, d
    return best


_GRADE = np.array([1.0 / 64, 1.0 / 16, 1.0 / 4, 1.0, 4.0, 16.0, 64.0, 256.0])


def inner(Q, r, lo, hi, func, n=24):
    """Integral over {r' in Q : lo < |r - r'| <= hi} of func(r') (func maps
    points [M, 3] to values [M, k]); see the module header."""
    Q = np.asarray(Q, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    a = closest_point(Q, r)
    C = float(np.dot(r - a, r - a))
    delta = math.sqrt(C)
    size = max(np.linalg.norm(Q[1] - Q[0]), np.linalg.norm(Q[2] - Q[1]), np.linalg.norm(Q[0] - Q[2]))
    if delta <= 1e-13 * size:  # r on Q up to rounding: the apex is r itself
        a, C, delta = r.copy(), 0.0, 0.0
    lo2 = lo * lo
    hi2 = hi * hi if np.isfinite(hi) else np.inf
    xn, wn = gl01(n)
    total = None
    for i in range(3):
        q1, q2 = Q[i], Q[(i + 1) % 3]
        two_a = np.linalg.norm(np.cross(q1 - a, q2 - a))
        if two_a <= 1e-13 * np.dot(q2 - q1, q2 - q1):
            continue  # the closest point lies on this edge: no fan triangle here
        e = q2 - q1
        g = q1 - r
        brk = [0.0, 1.0]
        # the fan triangle is thin where the apex is close to the far edge:
        # pieces graded around the foot of the apex on that edge's line
        ee = float(np.dot(e, e))
        vf = -float(np.dot(q1 - a, e)) / ee
        hf = float(np.linalg.norm(q1 - a + vf * e)) / math.sqrt(ee)
        for gk in (0.0, 0.25, 1.0, 4.0, 16.0):
            for v in (vf - gk * hf, vf + gk * hf):
                if 0.0 < v < 1.0:
                    brk.append(v)
        for x2 in (lo2, hi2):  # where the shell's bounding sphere crosses the far edge
            if not np.isfinite(x2) or x2 <= 0.0:
                continue
            A_, B_, C_ = np.dot(e, e), 2.0 * np.dot(g, e), np.dot(g, g) - x2
            disc = B_ * B_ - 4.0 * A_ * C_
            if disc > 0.0:
                sq = math.sqrt(disc)
                for v in ((-B_ - sq) / (2.0 * A_), (-B_ + sq) / (2.0 * A_)):
                    if 0.0 < v < 1.0:
                        brk.append(v)
        brk = np.sort(np.array(brk))
        for v0, v1 in zip(brk[:-1], brk[1:]):
            if v1 - v0 <= 0.0:
                continue
            v = v0 + (v1 - v0) * xn
            wv = (v1 - v0) * wn
            w = (q1 - a)[None, :] + v[:, None] * e[None, :]  # [nv, 3]
            A = np.einsum("ij,ij->i", w, w)
            B = w @ (r - a)

            def uroot(x2):
                if x2 <= C:
                    return np.zeros_like(A)
                if not np.isfinite(x2):
                    return np.full_like(A, np.inf)
                return (B + np.sqrt(B * B - A * (C - x2))) / A

            ulo = np.minimum(uroot(lo2), 1.0)
            uhi = np.minimum(uroot(hi2), 1.0)
            s = delta / np.sqrt(A)
            pts = np.concatenate([ulo[:, None], s[:, None] * _GRADE[None, :], uhi[:, None]], axis=1)
            pts = np.sort(np.clip(pts, ulo[:, None], np.maximum(uhi, ulo)[:, None]), axis=1)
            ua, ub = pts[:, :-1], pts[:, 1:]
            u = ua[:, :, None] + (ub - ua)[:, :, None] * xn[None, None, :]
            wu = (ub - ua)[:, :, None] * wn[None, None, :] * wv[:, None, None]
            u = np.where(wu > 0.0, u, 0.5)  # empty pieces (weight 0): any point off the apex
            rp = a[None, None, None, :] + u[..., None] * w[:, None, None, :]
            jac = two_a * u
            vals = func(rp.reshape(-1, 3))
            vals = vals.reshape(rp.shape[:3] + (-1,))
            part = np.einsum("abc,abck->k", wu * jac, vals)
            total = part if total is None else total + part
    return total


# ---------------------------------------------------------------- entries
class Mesh:
    """Geometry and tables of a mesh: vertices, triangles and the edge /
    BC tables of a topology object (edges, cells, fine triangles, BC
    fluxes), whose own tests pin them."""

    def __init__(self, topo):
        self.t = topo
        self.xyz = topo.xyz
        self.tri = topo.tri

    def coarse(self, c):
        return self.xyz[self.tri[c]]

    def fine(self, f):
        return self.t.fxyz[self.t.ftri[f]]

    def rwg_on(self, m):
        """[(triangle, field)] of RWG m: outward flux +1 through e_m from c+,
        -1 from c- (the unit-flux form of Sec. II-C)."""
        out = []
        v_minus, v_plus = self.t.edges[m]
        for c, sgn in ((self.t.cells[m, 0], 1.0), (self.t.cells[m, 1], -1.0)):
            verts = list(self.tri[c])
            opp = [k for k in range(3) if verts[k] not in (v_minus, v_plus)][0]
            fl = np.zeros(3)
            fl[opp] = sgn
            out.append((int(c), rt0(self.coarse(c), fl)))
        return out

    def bc_on(self, m):
        """[(fine triangle, field)] of BC function m from its tabulated fluxes."""
        out = []
        for f, lst in enumerate(self.t.bc_entries):
            for e, fl in lst:
                if e == m:
                    out.append((f, rt0(self.fine(f), fl)))
        return out


def _xw(R, lo, dt, xa):
    """the weight x^a, x = R/dt - lo/dt (1 without a time step)"""
    if not xa:
        return np.ones_like(R)
    return (R / dt - round(lo / dt)) ** xa


def v_shell(mesh, m, n, lo, hi, rule=None, dt=None, xa=0):
    """int int_{lo < R <= hi} f_m(r) . f_n(r') x^a / (4 pi R), f_m tested with
    the outer rule on its triangles (the orientation m outer, n inner); x =
    R/dt - j on shell j = lo/dt (a = 0: no weight)."""
    rule = rule or radon7_rule()
    tot = 0.0
    for c, fm in mesh.rwg_on(m):
        pts, w = rule_points(mesh.coarse(c), rule)
        fv = fm(pts)
        for cs, fn in mesh.rwg_on(n):
            Q = mesh.coarse(cs)
            for q in range(len(w)):
                r = pts[q]

                def f(rp, r=r, fn=fn):
                    R = np.linalg.norm(r - rp, axis=1)
                    return fn(rp) * (_xw(R, lo, dt, xa) / (FOUR_PI * R))[:, None]

                I = inner(Q, r, lo, hi, f)
                if I is not None:
                    tot += w[q] * float(np.dot(fv[q], I))
    return tot


def s_shell(mesh, c, cs, j, dt, rule=None):
    """int_c int_{c', shell j} x^p / (4 pi R), x = R/dt - j, p = 0, 1, 2, 3."""
    rule = rule or radon7_rule()
    pts, w = rule_points(mesh.coarse(c), rule)
    Q = mesh.coarse(cs)
    tot = np.zeros(4)
    for q in range(len(w)):
        r = pts[q]

        def f(rp, r=r):
            R = np.linalg.norm(r - rp, axis=1)
            x = R / dt - j
            return np.stack([np.ones_like(x), x, x * x, x * x * x], axis=1) / (FOUR_PI * R)[:, None]

        I = inner(Q, r, j * dt, (j + 1) * dt, f)
        if I is not None:
            tot += w[q] * I
    return tot


def n_shell(mesh, m, n, lo, hi, rule=None, dt=None, xa=0):
    """int int_{lo < R <= hi} g_m(r) . ((r - r') x f_n(r')) x^a / (4 pi R^3),
    g_m tested with the 3-point rule on its fine triangles; pairs whose fine
    test triangle lies in the source triangle are coplanar, where the
    integrand vanishes identically; x = R/dt - lo/dt (a = 0: no weight)."""
    rule = rule or three_point_rule()
    tot = 0.0
    for f, gm in mesh.bc_on(m):
        pts, w = rule_points(mesh.fine(f), rule)
        gv = gm(pts)
        for cs, fn in mesh.rwg_on(n):
            if mesh.t.fparent[f] == cs:
                continue
            Q = mesh.coarse(cs)
            for q in range(len(w)):
                r = pts[q]

                def k(rp, r=r, fn=fn):
                    d = r[None, :] - rp
                    R = np.linalg.norm(d, axis=1)
                    return np.cross(d, fn(rp)) * (_xw(R, lo, dt, xa) / (FOUR_PI * R ** 3))[:, None]

                I = inner(Q, r, lo, hi, k)
                if I is not None:
                    tot += w[q] * float(np.dot(gv[q], I))
    return tot


def _share_vertex(tri, c1, c2):
    return len(set(tri[c1]) & set(tri[c2])) > 0


def yukawa_bc_pair(mesh, m, n, kappa, src_rule=None):
    """int int g_m . g_n e^{-kappa R}/(4 pi R) over the fine triangles of the
    two BC functions, as the quadrature specification evaluates it: 3-point
    test rule; for fine triangles whose coarse parents share a vertex the
    static part 1/(4 pi R) integrated exactly (inner above) plus the bounded
    remainder (e^{-kappa R} - 1)/(4 pi R) by the 7-point source rule, for all
    other pairs the 7-point source rule on the whole kernel."""
    src_rule = src_rule or radon7_rule()
    tot = 0.0
    for f, gm in mesh.bc_on(m):
        pts, w = rule_points(mesh.fine(f), three_point_rule())
        gv = gm(pts)
        for fs, gn in mesh.bc_on(n):
            Q = mesh.fine(fs)
            near = _share_vertex(mesh.tri, mesh.t.fparent[f], mesh.t.fparent[fs])
            sp_, sw = rule_points(Q, src_rule)
            gs = gn(sp_)
            for q in range(len(w)):
                r = pts[q]
                R = np.linalg.norm(r - sp_, axis=1)
                if near:
                    I = inner(Q, r, 0.0, np.inf, lambda rp, r=r: gn(rp) / (FOUR_PI * np.linalg.norm(r - rp, axis=1))[:, None])
                    I = I + np.sum((sw * np.expm1(-kappa * R) / (FOUR_PI * R))[:, None] * gs, axis=0)
                else:
                    I = np.sum((sw * np.exp(-kappa * R) / (FOUR_PI * R))[:, None] * gs, axis=0)
                tot += w[q] * float(np.dot(gv[q], I))
    return tot


def yukawa_dual_pair(mesh, v, vs, kappa, src_rule=None):
    """sum over fine triangles t in the dual cell of v and t' in that of v' of
    int_t int_t' e^{-kappa R}/(4 pi R) / (A_t A_t'), evaluated as in
    yukawa_bc_pair (the scalar kernel of the hypersingular term, Sec. II-C)."""
    src_rule = src_rule or radon7_rule()
    tot = 0.0
    owner = mesh.t.fowner
    for f in np.nonzero(owner == v)[0]:
        P = mesh.fine(f)
        pts, w = rule_points(P, three_point_rule())
        for fs in np.nonzero(owner == vs)[0]:
            Q = mesh.fine(fs)
            near = _share_vertex(mesh.tri, mesh.t.fparent[f], mesh.t.fparent[fs])
            sp_, sw = rule_points(Q, src_rule)
            acc = 0.0
            for q in range(len(w)):
                r = pts[q]
                R = np.linalg.norm(r - sp_, axis=1)
                if near:
                    I = inner(Q, r, 0.0, np.inf, lambda rp, r=r: (1.0 / (FOUR_PI * np.linalg.norm(r - rp, axis=1)))[:, None])[0]
                    I += np.sum(sw * np.expm1(-kappa * R) / (FOUR_PI * R))
                else:
                    I = np.sum(sw * np.exp(-kappa * R) / (FOUR_PI * R))
                acc += w[q] * I
            tot += acc / (area(P) * area(Q))
    return tot


def mfie_pair(mesh, m, n, kappa, src_rule=None):
    """int int g_m . ((r - r') x f_n) (1 + kappa R) e^{-kappa R}/(4 pi R^3),
    BC test (3-point rule on fine triangles) against RWG trial (coarse), as
    the quadrature specification evaluates it: coplanar pairs zero; parents
    sharing a vertex: the static part 1/R^3 exactly (inner above) plus the
    remainder ((1 + kappa R) e^{-kappa R} - 1)/R^3 by the 7-point source
    rule; other pairs the 7-point source rule on the whole kernel."""
    src_rule = src_rule or radon7_rule()
    tot = 0.0
    for f, gm in mesh.bc_on(m):
        pts, w = rule_points(mesh.fine(f), three_point_rule())
        gv = gm(pts)
        for cs, fn in mesh.rwg_on(n):
            if mesh.t.fparent[f] == cs:
                continue
            Q = mesh.coarse(cs)
            near = _share_vertex(mesh.tri, mesh.t.fparent[f], cs)
            sp_, sw = rule_points(Q, src_rule)
            fs = fn(sp_)
            for q in range(len(w)):
                r = pts[q]
                d = r[None, :] - sp_
                R = np.linalg.norm(d, axis=1)
                x = kappa * R
                if near:
                    def k(rp, r=r):
                        dd = r[None, :] - rp
                        RR = np.linalg.norm(dd, axis=1)
                        return np.cross(dd, fn(rp)) / (FOUR_PI * RR ** 3)[:, None]
                    I = inner(Q, r, 0.0, np.inf, k)
                    rem = (np.expm1(-x) + x * np.exp(-x)) / R ** 3
                    I = I + np.sum((sw * rem / FOUR_PI)[:, None] * np.cross(d, fs), axis=0)
                else:
                    ker = (1.0 + x) * np.exp(-x) / R ** 3
                    I = np.sum((sw * ker / FOUR_PI)[:, None] * np.cross(d, fs), axis=0)
                tot += w[q] * float(np.dot(gv[q], I))
    return tot
