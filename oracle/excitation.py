"""Incident field and right-hand sides (oracle; test infrastructure).

Sec. II-C: e_m(t) = <n x f_m, n x e_in(t)> = int f_m . e_in ds and
h_m(t) = <n x g_m, n x h_in(t)> = int g_m . h_in ds (tangential fields).
Sec. V: h_in = eta^-1 k x e_in (eta = 1 here).
Sec. IV-A: r_k = -Z~ G^-T e~(t_k) + eta_c X~ G^-1 h(t_k), e~ = (dt~ P^{LH} + P^Sigma) e,
i.e. r_k = -P_E e(t_k) + P_M h(t_k) with the preconditioners of operators.py.

Pulses (reading of the configuration; the paper's own Gaussian is pulse 1):
  pulse 0: e = A p cos(2 pi f0 u) exp(-u^2 / (2 sig^2)), sig = 1/(2 pi bw)
  pulse 1: e = (4A/(w sqrt(pi))) p exp(-((4/w) u)^2)        (Sec. V)
  with u = t - t0 - k.r (c = 1).
Spatial quadrature: Radon 7-point rule on coarse (RWG) and fine (BC)
triangles.  Parity unpinned (the pulse-0 form is a reading).
"""
from __future__ import annotations

import numpy as np

from . import quadrature as Q


def pulse_value(wave, u):
    if wave.pulse == 0:
        sig = 1.0 / (2.0 * np.pi * wave.bw)
        return wave.amplitude * np.cos(2.0 * np.pi * wave.f0 * u) * np.exp(-u * u / (2.0 * sig * sig))
    w = wave.w
    return (4.0 * wave.amplitude / (w * np.sqrt(np.pi))) * np.exp(-((4.0 / w) * u) ** 2)


def incident_e(wave, r, t):
    """e_in at points r [..., 3] and scalar time t -> [..., 3]."""
    k = np.asarray(wave.k_hat, dtype=np.float64)
    p = np.asarray(wave.pol, dtype=np.float64)
    u = t - wave.t0 - r @ k
    return pulse_value(wave, u)[..., None] * p


def incident_h(wave, r, t):
    k = np.asarray(wave.k_hat, dtype=np.float64)
    return np.cross(k, incident_e(wave, r, t))


def _testing_matrices(asm):
    """Sparse maps from field samples at the quadrature points to the tested
    values: e = We @ E_samples, h = Wh @ H_samples (samples flattened as
    [triangle, point, xyz])."""
    import scipy.sparse as sp
    t = asm.topo
    bary, w = Q.radon7()
    Pc = t.xyz[t.tri]
    pts_c = np.einsum("qi,cik->cqk", bary, Pc)
    rows, cols, vals = [], [], []
    for c in range(t.nc):
        for b in range(3):
            f = t.tri_sign[c, b] * (pts_c[c] - Pc[c, b]) / (2.0 * t.area[c])
            for q in range(7):
                for k in range(3):
                    rows.append(t.tri_edge[c, b])
                    cols.append((c * 7 + q) * 3 + k)
                    vals.append(t.area[c] * w[q] * f[q, k])
    We = sp.csr_matrix((vals, (rows, cols)), shape=(t.ne, t.nc * 21))
    Pf = t.fxyz[t.ftri]
    pts_f = np.einsum("qi,cik->cqk", bary, Pf)
    rows, cols, vals = [], [], []
    for ft, lst in enumerate(t.bc_entries):
        A = t.farea[ft]
        P = Pf[ft]
        for e, fl in lst:
            g = sum(fl[i] * (pts_f[ft] - P[i]) for i in range(3)) / (2.0 * A)
            for q in range(7):
                for k in range(3):
                    rows.append(e)
                    cols.append((ft * 7 + q) * 3 + k)
                    vals.append(A * w[q] * g[q, k])
    Wh = sp.csr_matrix((vals, (rows, cols)), shape=(t.ne, len(Pf) * 21))
    return We, pts_c.reshape(-1, 3), Wh, pts_f.reshape(-1, 3)


def tested_fields(asm, wave, n_steps: int):
    """e(t_k), h(t_k) for k = 1..n_steps -> arrays [n_steps, ne]."""
    if not hasattr(asm, "_testing"):
        asm._testing = _testing_matrices(asm)
    We, pc, Wh, pf = asm._testing
    e_out = np.zeros((n_steps, asm.topo.ne))
    h_out = np.zeros((n_steps, asm.topo.ne))
    for s in range(n_steps):
        tk = (s + 1) * asm.dt
        e_out[s] = We @ incident_e(wave, pc, tk).reshape(-1)
        h_out[s] = Wh @ incident_h(wave, pf, tk).reshape(-1)
    return e_out, h_out


def rhs(asm, wave, n_steps: int):
    e, h = tested_fields(asm, wave, n_steps)
    return -(e @ asm.PE.T) + h @ asm.PM.T
