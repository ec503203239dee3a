"""Operator assembly of the qHP TD-CFIE (oracle; test infrastructure).

Normalised units: c = 1 (time measured in metres of c*t), eta = 1, so
T0 = D (diameter), kappa = 1/dt, dt~ = dt/D.

Sections followed:
  * Sec. II-C     Gram G_mn = <n x g_m, f_n>; Yukawa Z^s, Z^h (BC-BC) and M
                  (BC test, RWG trial) with wave number -j kappa, kappa = 1/(c dt)
                  (Sec. II-B).
  * Sec. II-D     projectors P^Sigma = Sigma (Sigma^T Sigma)^+ Sigma^T,
                  P^{Lambda H} = I - P^Sigma, PP^Lambda = Lambda (Lambda^T Lambda)^+
                  Lambda^T, PP^{Sigma H} = I - PP^Lambda.
  * Sec. III-B    Z~ = (dt~ PP^{SH} + PP^L) Z (PP^{SH} + dt~^-1 PP^L).
  * Sec. III-C    X = G/2 - M, X~ = (dt~ PP^{SH} + PP^L) X.
  * Sec. IV       coupling (eq. qHP_TDCFIE) and the blocks T_k of eq.
                  dis_TD_CFIE:  T_k = Z~ G^-T Z~_k + eta_c X~ G^-1 X~_k, with the
                  stabilised operators applied to (h_0 P^{LH} + q_0 P^Sigma) and
                  tested at t = k dt (reading: the printed index places the
                  trial function at i dt and tests at 0, i.e. lag i; T_k
                  multiplies y_{i-k} in the marching formula).

Derived lag matrices (substituting the temporal bases of Sec. IV-A into the
operators of Sec. II-A; shell j is j dt < R <= (j+1) dt, pieces of h_0, q_0
taken on half-open intervals so each point pair falls in one shell):
  A_k = -(V_k - V_{k-1})/dt                       (T^s on h_0, tested at k dt)
  B_k = -T0 Sigma diag(1/A) Sq_k diag(1/A) Sigma^T    (d~_t T^h on q_0)
        Sq_k = 1/2(S_k^0 - 2 S_k^1 + S_k^2) + (1/2 S_{k-1}^0 + S_{k-1}^1 - S_{k-1}^2)
               + 1/2 S_{k-2}^2       (q_0 on the three shells it spans)
  C_k = G/2 delta_k0 + (k+1) N_k + (1-k) N_{k-1}    (G/2 + K on h_0)
  W^E_k = A_k P^{LH} + (A_k - A_{k-1})/dt~ P^Sigma + B_k
  W^M_k = C_k P^{LH} + (C_k - C_{k-1})/dt~ P^Sigma
  T_k = P_E W^E_k + P_M W^M_k,  P_E = Z~ G^-T (dt~ P^{LH} + P^Sigma),
                                P_M = eta_c X~ G^-1
The identity d~_t q_i = (h_i - h_{i+1})/dt~ (Remark of Sec. IV-B) turns the
q-basis vector-potential and MFIE terms into the h-basis differences above.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import scipy.linalg as sla

from . import quadrature as Q
from .topology import Topology

FOUR_PI = 4.0 * math.pi


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def n_lags(diameter: float, dt: float, order: int = 1) -> int:
    """K such that T_k = 0 for k > K: q_0 of temporal order p spans p + 2
    intervals, so it reaches p + 1 shells past the largest distance D.  A 1e-9
    relative guard makes D/dt that is an integer up to rounding give the same
    K on every platform."""
    return int(math.ceil(diameter / dt - 1e-9)) + int(order)


def pinv_laplacian(L: np.ndarray) -> np.ndarray:
    """Moore-Penrose pseudo-inverse of the Laplacian of a connected graph:
    (L + 11^T/n)^-1 - 11^T/n (the null space of L is span{1})."""
    n = L.shape[0]
    J = np.full((n, n), 1.0 / n)
    return np.linalg.inv(L + J) - J



def h0_prime_combine(Vk, Vk1, dt):
    """-int int f.f h_0'(k dt - R)/(4 pi R): h_0' is +1/dt for R in shell k
    and -1/dt for R in shell k-1 (T^s carries -eta/c = -1)."""
    return -(Vk - Vk1) / dt


def q0_combine(Sk, Sk1, Sk2):
    """int int q_0(k dt - R)/(4 pi R) from the x-moments (x = R/dt - j) of
    shells k, k-1, k-2: q_0 = (1-x)^2/2, 1/2 + x - x^2, x^2/2 there
    (Sec. IV-A definition of q_0 with tau/dt = -x, 1-x, 2-x)."""
    return (0.5 * (Sk[0] - 2.0 * Sk[1] + Sk[2])
            + (0.5 * Sk1[0] + Sk1[1] - Sk1[2])
            + 0.5 * Sk2[2])


def mfie_combine(Nk, Nk1, k):
    """K on h_0 tested at k dt: the kernel h_0(tau)/R^2 + h_0'(tau)/(cR)
    equals (h_0(tau) + R h_0'(tau)) / R^2, which is k+1 on shell k and 1-k on
    shell k-1."""
    return (k + 1.0) * Nk + (1.0 - k) * Nk1


class Projectors:
    """Quasi-Helmholtz projectors of Sec. II-D, dense FP64."""

    def __init__(self, topo: Topology):
        S = topo.Sigma.toarray()
        L = topo.Lambda.toarray()
        self.LS_pinv = pinv_laplacian(S.T @ S)
        self.LL_pinv = pinv_laplacian(L.T @ L)
        self.PS = S @ self.LS_pinv @ S.T
        self.PLH = np.eye(topo.ne) - self.PS
        self.PPL = L @ self.LL_pinv @ L.T
        self.PPSH = np.eye(topo.ne) - self.PPL


class Assembly:
    """Everything the marching scheme needs, for one mesh and time step."""

    def __init__(self, xyz, tri, dt: float, spec: Q.Spec | None = None, eta_c: float = 1.0,
                 K: int | None = None, order: int = 1):
        self.topo = t = Topology(xyz, tri)
        self.dt = float(dt)
        self.D = t.diameter
        self.T0 = self.D  # D / c with c = 1
        self.dtn = self.dt / self.T0  # dt~
        self.kappa = 1.0 / self.dt  # kappa = 1/(c dt)
        self.eta_c = float(eta_c)
        self.spec = spec or Q.Spec()
        if order not in (1, 2):
            raise ValueError("temporal order 1 (hat functions) or 2 (quadratic interpolators)")
        self.order = int(order)
        self.K = n_lags(self.D, self.dt, self.order) if K is None else int(K)
        self.n_shells = self.K
        self.proj = Projectors(t)
        self._bc_arrays()

    # ------------------------------------------------------------ tables
    def _bc_arrays(self):
        t = self.topo
        off = [0]
        edge, flux = [], []
        for lst in t.bc_entries:
            for e, fl in lst:
                edge.append(e)
                flux.append(fl)
            off.append(len(edge))
        self.bc_off = _i64(off)
        self.bc_edge = _i64(edge)
        self.bc_flux = _f64(np.array(flux).reshape(-1, 3))

    # ------------------------------------------------------------ Gram
    def gram(self, rule=None) -> np.ndarray:
        """G_mn = int (n x g_m) . f_n, exact with the degree-2 rule on each
        fine triangle (both factors are linear there)."""
        t = self.topo
        G = np.zeros((t.ne, t.ne))
        bary, w = rule or Q.tri3()
        for ft in range(6 * t.nc):
            c = t.fparent[ft]
            P = t.fxyz[t.ftri[ft]]
            A = t.farea[ft]
            pts = bary @ P
            n = t.normal[c]
            Pc = t.xyz[t.tri[c]]
            for e, fl in t.bc_entries[ft]:
                g = sum(fl[i] * (pts - P[i]) for i in range(3)) / (2.0 * A)
                ng = np.cross(n, g)
                for b in range(3):
                    f = t.tri_sign[c, b] * (pts - Pc[b]) / (2.0 * t.area[c])
                    G[e, t.tri_edge[c, b]] += A * np.sum(w * np.einsum("qk,qk->q", ng, f))
        return G

    # ------------------------------------------------------------ Yukawa
    def yukawa(self):
        """Z^s, Z^h and M of Sec. II-C with kappa = 1/dt (eta = 1).
        Z^s = -kappa int int g.g G_k,  Z^h = -(1/kappa) int int div g div g G_k,
        M = int int g.((r - r') x f)(1 + kappa R) e^{-kappa R}/(4 pi R^3)."""
        return self._yukawa(self.kappa)

    def _yukawa(self, kappa: float):
        t, s = self.topo, self.spec
        L = Q.lib()
        nf = 6 * t.nc
        Zs = np.zeros((t.ne, t.ne))
        D = np.zeros((t.nv, t.nv))
        fb, fw = _f64(s.fine_rule[0]), _f64(s.fine_rule[1])
        sb, sw = _f64(s.src_rule[0]), _f64(s.src_rule[1])
        gx, gw = _f64(s.gx), _f64(s.gw)
        fxyz, ftri, fpar, fown = _f64(t.fxyz), _i64(t.ftri), _i64(t.fparent), _i64(t.fowner)
        tri = _i64(t.tri)
        L.orc_static_bcbc.restype = None
        L.orc_static_bcbc(_ptr(fxyz), _ptr(ftri), ctypes.c_long(nf), _ptr(fpar), _ptr(fown),
                          _ptr(tri), _ptr(self.bc_off), _ptr(self.bc_edge), _ptr(self.bc_flux),
                          ctypes.c_long(t.ne), ctypes.c_long(t.nv), ctypes.c_double(kappa),
                          ctypes.c_int(len(fw)), _ptr(fb), _ptr(fw), ctypes.c_int(len(sw)),
                          _ptr(sb), _ptr(sw), ctypes.c_int(len(gx)), _ptr(gx), _ptr(gw),
                          _ptr(Zs), _ptr(D))
        M = np.zeros((t.ne, t.ne))
        xyz, te, ts = _f64(t.xyz), _i64(t.tri_edge), _i64(t.tri_sign)
        L.orc_static_mfie.restype = None
        L.orc_static_mfie(_ptr(fxyz), _ptr(ftri), ctypes.c_long(nf), _ptr(fpar),
                          _ptr(self.bc_off), _ptr(self.bc_edge), _ptr(self.bc_flux),
                          _ptr(xyz), _ptr(tri), ctypes.c_long(t.nc), _ptr(te), _ptr(ts),
                          ctypes.c_long(t.ne), ctypes.c_double(kappa), ctypes.c_int(len(fw)),
                          _ptr(fb), _ptr(fw), ctypes.c_int(len(sw)), _ptr(sb), _ptr(sw),
                          ctypes.c_int(len(gx)), _ptr(gx), _ptr(gw),
                          ctypes.c_double(s.coplanar_tol), _ptr(M))
        Zs = 0.5 * (Zs + Zs.T)  # Galerkin symmetry of the BC-BC pairing
        D = 0.5 * (D + D.T)
        # div g_m on fine t in the dual cell of v is -Lambda_mv / (2 N_v A_t)
        Lam = t.Lambda.toarray()
        inv2n = 1.0 / (2.0 * t.valence)
        Lw = Lam * inv2n[None, :]
        Zh_int = Lw @ D @ Lw.T
        Zs_op = -kappa * Zs
        Zh_op = -(1.0 / kappa) * Zh_int
        return Zs_op, Zh_op, M

    def static_mfie(self):
        """M_0 (kappa = 0), used by the static-property pin."""
        return self._mfie_only(0.0)

    def _mfie_only(self, kappa):
        t, s = self.topo, self.spec
        L = Q.lib()
        nf = 6 * t.nc
        M = np.zeros((t.ne, t.ne))
        fb, fw = _f64(s.fine_rule[0]), _f64(s.fine_rule[1])
        sb, sw = _f64(s.src_rule[0]), _f64(s.src_rule[1])
        gx, gw = _f64(s.gx), _f64(s.gw)
        L.orc_static_mfie.restype = None
        L.orc_static_mfie(_ptr(_f64(t.fxyz)), _ptr(_i64(t.ftri)), ctypes.c_long(nf),
                          _ptr(_i64(t.fparent)), _ptr(self.bc_off), _ptr(self.bc_edge),
                          _ptr(self.bc_flux), _ptr(_f64(t.xyz)), _ptr(_i64(t.tri)),
                          ctypes.c_long(t.nc), _ptr(_i64(t.tri_edge)), _ptr(_i64(t.tri_sign)),
                          ctypes.c_long(t.ne), ctypes.c_double(kappa), ctypes.c_int(len(fw)),
                          _ptr(fb), _ptr(fw), ctypes.c_int(len(sw)), _ptr(sb), _ptr(sw),
                          ctypes.c_int(len(gx)), _ptr(gx), _ptr(gw),
                          ctypes.c_double(s.coplanar_tol), _ptr(M))
        return M

    # ------------------------------------------------------------ retarded
    def shells(self):
        """Shell moments V_j, S_j^p (coarse) and N_j (BC x RWG), j < n_shells.
        Order 1: V [nsh][ne][ne], S [nsh][3][nc][nc], N [nsh][ne][ne].  Higher
        orders p: the x^a moments V [nsh][p][ne][ne] (a < p), S [nsh][p+2] and
        N [nsh][p+1][ne][ne] (see temporal.py)."""
        t, s = self.topo, self.spec
        L = Q.lib()
        nsh, p = self.n_shells, self.order
        V = np.zeros((nsh, p, t.ne, t.ne))
        S = np.zeros((nsh, p + 2, t.nc, t.nc))
        cb, cw = _f64(s.coarse_rule[0]), _f64(s.coarse_rule[1])
        gx, gw = _f64(s.gx), _f64(s.gw)
        xyz, tri, te, ts = _f64(t.xyz), _i64(t.tri), _i64(t.tri_edge), _i64(t.tri_sign)
        L.orc_retarded_coarse.restype = None
        L.orc_retarded_coarse(_ptr(xyz), _ptr(tri), ctypes.c_long(t.nc), _ptr(te), _ptr(ts),
                              ctypes.c_long(t.ne), ctypes.c_double(self.dt), ctypes.c_long(nsh),
                              ctypes.c_int(p), ctypes.c_int(len(cw)), _ptr(cb), _ptr(cw), ctypes.c_int(len(gx)),
                              _ptr(gx), _ptr(gw), _ptr(V), _ptr(S))
        V = 0.5 * (V + V.transpose(0, 1, 3, 2))
        S = 0.5 * (S + S.transpose(0, 1, 3, 2))
        N = np.zeros((nsh, p + 1, t.ne, t.ne))
        fb, fw = _f64(s.fine_rule[0]), _f64(s.fine_rule[1])
        L.orc_retarded_bc.restype = None
        L.orc_retarded_bc(_ptr(_f64(t.fxyz)), _ptr(_i64(t.ftri)), ctypes.c_long(6 * t.nc),
                          _ptr(_i64(t.fparent)), _ptr(self.bc_off), _ptr(self.bc_edge),
                          _ptr(self.bc_flux), _ptr(xyz), _ptr(tri), ctypes.c_long(t.nc),
                          _ptr(te), _ptr(ts), ctypes.c_long(t.ne), ctypes.c_double(self.dt),
                          ctypes.c_long(nsh), ctypes.c_int(p), ctypes.c_int(len(fw)), _ptr(fb), _ptr(fw),
                          ctypes.c_int(len(gx)), _ptr(gx), _ptr(gw),
                          ctypes.c_double(s.coplanar_tol), _ptr(N))
        if p == 1:
            return V[:, 0], S, N[:, 0]
        return V, S, N

    def lag_matrices(self, V, S, N, G):
        """Raw lag matrices A_k, B_k, C_k for k = 0..K (see module header)."""
        if self.order != 1:
            return self.lag_matrices_order(V, S, N, G)
        t = self.topo
        K = self.K

        def sh(X, j):
            return X[j] if 0 <= j < X.shape[0] else np.zeros(X.shape[1:])

        Sig = t.Sigma.toarray()
        SA = Sig * (1.0 / t.area)[None, :]
        A, B, C = [], [], []
        for k in range(K + 1):
            A.append(h0_prime_combine(sh(V, k), sh(V, k - 1), self.dt))
            Sq = q0_combine(sh(S, k), sh(S, k - 1), sh(S, k - 2))
            B.append(-self.T0 * SA @ Sq @ SA.T)
            Ck = mfie_combine(sh(N, k), sh(N, k - 1), k)
            if k == 0:
                Ck = Ck + 0.5 * G
            C.append(Ck)
        return A, B, C

    def lag_matrices_order(self, V, S, N, G, order=None):
        """Raw lag matrices for temporal bases of order p (temporal.py): sums
        of the x^a shell moments with the coefficients of h_0', q_0 and
        h_0 + R h_0' on the interval each shell falls in.  V [nsh][p], S
        [nsh][p+2], N [nsh][p+1] moment-major (for p = 1 also the plain
        arrays of `shells`)."""
        from . import temporal
        t = self.topo
        K, p = self.K, int(order or self.order)
        if V.ndim == 3:
            V, N = V[:, None], N[:, None]
        da, qa, ca = temporal.combos(p)
        Sig = t.Sigma.toarray()
        SA = Sig * (1.0 / t.area)[None, :]
        zV, zS = np.zeros(V.shape[2:]), np.zeros(S.shape[2:])

        def sh(X, j, a, z):
            return X[j, a] if 0 <= j < X.shape[0] and a < X.shape[1] else z

        A, B, C = [], [], []
        for k in range(K + 1):
            Ak = zV.copy()
            Ck = 0.5 * G if k == 0 else zV.copy()
            for m in range(p + 1):
                cam = ca(k, m)
                for a in range(p):
                    Ak = Ak - (da[m][a] / self.dt) * sh(V, k - m, a, zV)
                for a in range(p + 1):
                    Ck = Ck + cam[a] * sh(N, k - m, a, zV)
            Sq = zS.copy()
            for m in range(p + 2):
                for a in range(p + 2):
                    Sq = Sq + qa[m][a] * sh(S, k - m, a, zS)
            A.append(Ak)
            B.append(-self.T0 * SA @ Sq @ SA.T)
            C.append(Ck)
        return A, B, C

    # ------------------------------------------------------------ combine
    def preconditioners(self, G, Zs, Zh, M):
        """P_E = Z~ G^-T (dt~ P^{LH} + P^Sigma) and P_M = eta_c X~ G^-1."""
        p, dtn = self.proj, self.dtn
        left = dtn * p.PPSH + p.PPL
        Zt = left @ Zs @ (p.PPSH + p.PPL / dtn) + (1.0 / dtn) * p.PPL @ Zh @ p.PPL
        X = 0.5 * G - M
        Xt = left @ X
        Gi = np.linalg.inv(G)
        PE = Zt @ Gi.T @ (dtn * p.PLH + p.PS)
        PM = self.eta_c * Xt @ Gi
        self.Zt, self.Xt = Zt, Xt
        return PE, PM

    def slabs(self, PE, PM, A, B, C):
        p, dtn = self.proj, self.dtn
        T = []
        for k in range(self.K + 1):
            Ak1 = A[k - 1] if k > 0 else np.zeros_like(A[0])
            Ck1 = C[k - 1] if k > 0 else np.zeros_like(C[0])
            WE = A[k] @ p.PLH + (A[k] - Ak1) / dtn @ p.PS + B[k]
            WM = C[k] @ p.PLH + (C[k] - Ck1) / dtn @ p.PS
            T.append(PE @ WE + PM @ WM)
        return np.array(T)

    def build(self):
        """Full assembly: returns the slabs T [K+1, ne, ne] and keeps the
        intermediate operators as attributes."""
        self.G = self.gram()
        self.Zs, self.Zh, self.M = self.yukawa()
        self.PE, self.PM = self.preconditioners(self.G, self.Zs, self.Zh, self.M)
        self.V, self.S, self.N = self.shells()
        self.A, self.B, self.C = self.lag_matrices(self.V, self.S, self.N, self.G)
        self.T = self.slabs(self.PE, self.PM, self.A, self.B, self.C)
        return self.T
