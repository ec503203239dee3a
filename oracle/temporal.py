"""Temporal basis pairs (h_0, q_0) of order p (oracle; test infrastructure).

Sec. IV-A discretises the solenoidal part of the auxiliary unknown with the
hat functions h_i and the irrotational part with q_i; the Remark of Sec. IV-B
allows shifted piecewise-polynomial Lagrange interpolators of higher order for
h_i, with q_i chosen so that q_i' = (h_i - h_{i+1})/dt.

Reading (the paper fixes only the identity): h_0 of order p is, on each
interval [(m-1) dt, m dt), m = 0..p, the Lagrange polynomial through the p+1
nodes (m-p) dt, ..., m dt that is 1 at t = 0 and 0 at the others (the
interpolation uses the latest sample and the p before it); zero elsewhere.
p = 1 is the hat function.  q_0(t) = int_{-inf}^t (h_0(s) - h_0(s - dt))/dt ds,
on [(m-1) dt, m dt) for m = 0..p+1.

In units u = t/dt.  For a source point at distance R in shell j (j dt < R <=
(j+1) dt, x = R/dt - j in (0, 1]) tested at t = k dt the retarded time
k dt - R lies in interval m = k - j at u = m - x, so every piece becomes a
polynomial in x and the lag matrices are sums of the x^a shell moments:

  A_k = -(1/dt) sum_m sum_a da[m][a] V_{k-m}^(a)        (h_0', a <= p-1)
  Sq_k = sum_m sum_a qa[m][a] S_{k-m}^(a)               (q_0,  a <= p+1)
  C_k = G/2 delta_k0 + sum_m sum_a ca(k,m)[a] N_{k-m}^(a)  (h_0 + R h_0', a <= p)

with h_0 + R h_0' the MFIE kernel's time dependence (h(tau)/R^3 + h'(tau)/R^2,
R = (j + x) dt).  For p = 1 these reduce to -(V_k - V_{k-1})/dt,
1/2(S^0 - 2S^1 + S^2)_k + (1/2 S^0 + S^1 - S^2)_{k-1} + 1/2 S^2_{k-2} and
(k+1) N_k + (1-k) N_{k-1}.
"""
from __future__ import annotations

from numpy.polynomial import polynomial as P
import numpy as np


def h0_pieces(p: int) -> list[np.ndarray]:
    """Coefficients (ascending powers of u) of h_0 on [m-1, m), m = 0..p."""
    out = []
    for m in range(p + 1):
        c = np.array([1.0])
        for n in range(m - p, m + 1):
            if n != 0:
                c = P.polymul(c, np.array([-n, 1.0]) / (0.0 - n))
        out.append(c)
    return out


def _shift(c: np.ndarray, s: float) -> np.ndarray:
    """Coefficients of c(u - s)."""
    out = np.zeros(1)
    base = np.array([-s, 1.0])
    for a, ca in enumerate(c):
        out = P.polyadd(out, ca * P.polypow(base, a))
    return out


def q0_pieces(p: int) -> list[np.ndarray]:
    """Coefficients of q_0 on [m-1, m), m = 0..p+1: the integral from u = -1
    of h_0(v) - h_0(v - 1) (h_0(v - 1) is h_0's piece m - 1 shifted by one)."""
    h = h0_pieces(p)
    out, left = [], 0.0
    for m in range(p + 2):
        g = h[m] if m <= p else np.zeros(1)
        if m >= 1:
            g = P.polysub(g, _shift(h[m - 1], 1.0))
        G = P.polyint(g)
        G = P.polyadd(G, np.array([left - P.polyval(m - 1.0, G)]))  # continuous at u = m - 1
        out.append(G)
        left = P.polyval(float(m), G)
    return out


def in_x(c: np.ndarray, m: int) -> np.ndarray:
    """Coefficients in x of c(u) at u = m - x."""
    out = np.zeros(1)
    base = np.array([float(m), -1.0])
    for a, ca in enumerate(c):
        out = P.polyadd(out, ca * P.polypow(base, a))
    return out


def _pad(c: np.ndarray, n: int) -> np.ndarray:
    out = np.zeros(n)
    out[:min(n, len(c))] = c[:n]
    return out


def combos(p: int):
    """(da, qa, ca): da[m] (m = 0..p, length p) the x-coefficients of dh_0/du,
    qa[m] (m = 0..p+1, length p+2) those of q_0, and ca(k, m) (length p+1)
    those of h_0 + R h_0' for lag k and interval m (R/dt = k - m + x)."""
    h = h0_pieces(p)
    da = [_pad(in_x(P.polyder(h[m]), m), p) for m in range(p + 1)]
    qa = [_pad(in_x(c, m), p + 2) for m, c in enumerate(q0_pieces(p))]

    def ca(k: int, m: int) -> np.ndarray:
        hx = in_x(h[m], m)
        dx = in_x(P.polyder(h[m]), m)
        return _pad(P.polyadd(hx, P.polymul(np.array([float(k - m), 1.0]), dx)), p + 1)

    return da, qa, ca


def h0(p: int, u: float) -> float:
    """h_0 at u = t/dt."""
    if not (-1.0 <= u < p):
        return 0.0
    m = int(np.floor(u)) + 1
    return float(P.polyval(u, h0_pieces(p)[m]))


def q0(p: int, u: float) -> float:
    """q_0 at u = t/dt."""
    if u < -1.0:
        return 0.0
    if u >= p + 1:
        return float(P.polyval(float(p + 1), q0_pieces(p)[p + 1]))
    m = int(np.floor(u)) + 1
    return float(P.polyval(u, q0_pieces(p)[m]))
