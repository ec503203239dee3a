"""Quadrature rules and the Python driver of the C quadrature core (oracle).

The paper states no quadrature rule, singular-integral scheme or treatment of
the piecewise temporal kernels (Sec. IV-A only fixes the temporal bases).  The
project fixes one written specification, implemented separately here (plain C
in ``quad_oracle.c``) and in the HIP library:

* Test (outer) integrals: symmetric triangle rules -- Radon's 7-point degree-5
  rule on coarse triangles, the 3-point degree-2 rule (points (2/3,1/6,1/6))
  on fine (barycentric) triangles.
* Source (inner) integrals with a 1/R, R^p/R or (r-r')/R^3 kernel restricted
  to a distance shell jdt < R <= (j+1)dt: integrated in polar coordinates
  about the projection p of the test point onto the source plane, with closed
  forms in the radial variable and n_psi-point Gauss-Legendre in the angle,
  taken in the variable s = asinh(t/h) along each edge (t the coordinate along
  the edge line, h the distance of p to it), on every sub-interval between the
  points where a shell circle crosses the edge; on sub-intervals where the
  shell lies wholly inside the edge's wedge the angular integrals are exact.
* Yukawa kernels e^{-kR}/(4 pi R) and (1+kR)e^{-kR}/(4 pi R^2): on pairs whose
  coarse parent triangles share a vertex, the static (k = 0) part goes through
  the polar scheme above and the bounded remainder through a 7-point source
  product rule; all other pairs use the product rule for the whole kernel.
* MFIE kernel pairs with the fine test triangle inside the coarse source
  triangle contribute zero (the integrand vanishes on coplanar pairs), as do
  test points within 1e-12 * (source edge length) of the source plane.

Parity unpinned as a whole: the specification is a reading, not the paper's.
Its parts are pinned by the tests (exact monomials, annulus closed forms,
the closed-form flat-triangle potential, convergence in n_psi).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "quad_oracle.c")
_LIB = os.path.join(_HERE, "_quad_oracle.so")


def radon7():
    """Radon's 7-point, degree-5 rule on the triangle: barycentric points and
    weights (summing to 1)."""
    s15 = np.sqrt(15.0)
    a1, b1 = (9.0 - 2.0 * s15) / 21.0, (6.0 + s15) / 21.0
    a2, b2 = (9.0 + 2.0 * s15) / 21.0, (6.0 - s15) / 21.0
    w1, w2 = (155.0 + s15) / 1200.0, (155.0 - s15) / 1200.0
    bary = [[1 / 3, 1 / 3, 1 / 3],
            [a1, b1, b1], [b1, a1, b1], [b1, b1, a1],
            [a2, b2, b2], [b2, a2, b2], [b2, b2, a2]]
    w = [9.0 / 40.0] + [w1] * 3 + [w2] * 3
    return np.array(bary), np.array(w)


def tri3():
    """3-point, degree-2 interior rule."""
    bary = [[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]]
    return np.array(bary), np.array([1 / 3, 1 / 3, 1 / 3])


def gauss_legendre(n: int):
    x, w = np.polynomial.legendre.leggauss(int(n))
    return x, w


def build_c(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c99", "-o", _LIB, _SRC, "-lm"]
        subprocess.check_call(cmd)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build_c())
    return _lib


def _p(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


class Spec:
    """Quadrature parameters shared by the whole assembly."""

    def __init__(self, n_psi: int = 10, coarse_rule=None, fine_rule=None, src_rule=None,
                 coplanar_tol: float = 1e-12):
        self.n_psi = n_psi
        self.coarse_rule = coarse_rule or radon7()
        self.fine_rule = fine_rule or tri3()
        self.src_rule = src_rule or radon7()
        self.coplanar_tol = coplanar_tol
        self.gx, self.gw = gauss_legendre(n_psi)


def inner_moments(P, r, s_lo, s_hi, j_shell, dt, spec: Spec):
    """Single inner integral over triangle P (3x3) from test point r on the
    radial segment s_lo < R <= s_hi (s_hi = inf for all of the triangle).
    Returns dict with I0 = int 1/R, Iu = int (r'-p)/R, Sx[p] = int x^p/R
    (x = R/dt - j_shell), W = int (r - r')/R^3 (0 on coplanar points)."""
    L = lib()
    P, pP = _p(P, np.float64)
    r, pr = _p(r, np.float64)
    out = np.zeros(10)
    _, po = _p(out, np.float64)
    gx, pgx = _p(spec.gx, np.float64)
    gw, pgw = _p(spec.gw, np.float64)
    L.orc_inner.restype = None
    L.orc_inner(pP, pr, ctypes.c_double(s_lo), ctypes.c_double(s_hi), ctypes.c_double(j_shell),
                ctypes.c_double(dt), ctypes.c_int(len(gx)), pgx, pgw,
                ctypes.c_double(spec.coplanar_tol), po)
    return {"I0": out[0], "Iu": out[1:4].copy(), "Sx": out[4:7].copy(), "W": out[7:10].copy()}
