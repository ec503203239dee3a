"""Pins of the oracle's quadrature: rules, shell integrals, static potential.

The paper fixes no quadrature; these pins tie the oracle's written
specification to closed forms that do not depend on it."""
import math

import numpy as np
import pytest

from oracle import quadrature as Q


@pytest.mark.parametrize("rule,deg", [(Q.radon7, 5), (Q.tri3, 2)])
def test_triangle_rules_exact(rule, deg):
    bary, w = rule()
    assert abs(w.sum() - 1.0) < 1e-15
    x, y = bary[:, 1], bary[:, 2]  # reference triangle (0,0),(1,0),(0,1), area 1/2
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(0.5 * np.sum(w * x ** a * y ** b) - exact) < 1e-15
    # one degree higher is not exact for at least one monomial
    errs = []
    for a in range(deg + 2):
        b = deg + 1 - a
        exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
        errs.append(abs(0.5 * np.sum(w * x ** a * y ** b) - exact))
    assert max(errs) > 1e-6


BIG = np.array([[-10.0, -10.0, 0.0], [20.0, -10.0, 0.0], [-10.0, 20.0, 0.0]])


@pytest.mark.parametrize("d", [0.0, 0.3, -0.2])
@pytest.mark.parametrize("seg", [(0.0, 0.5), (0.5, 0.9), (0.35, 0.37), (1.0, 4.0)])
def test_annulus_closed_forms(d, seg):
    """Shell integrals over a triangle that contains the whole annulus: the
    polar Jacobian gives 2 pi times one-dimensional integrals in R."""
    spec = Q.Spec(n_psi=6)
    r = np.array([0.1, 0.2, d])
    a, b = seg
    dt, j = 0.25, 3
    o = Q.inner_moments(BIG, r, a, b, j, dt, spec)
    lo = max(a, abs(d))
    if b <= lo:
        assert o["I0"] == 0.0
        return
    assert abs(o["I0"] - 2 * np.pi * (b - lo)) < 1e-13
    for p in range(3):
        ex = 2 * np.pi * dt * ((b / dt - j) ** (p + 1) - (lo / dt - j) ** (p + 1)) / (p + 1)
        assert abs(o["Sx"][p] - ex) < 1e-12 * max(1.0, abs(ex))
    assert np.abs(o["Iu"]).max() < 1e-11 * max(1.0, b * b)  # symmetric about p (angular quadrature)
    # W = int (r - r')/R^3: only the normal part survives, 2 pi d (1/lo - 1/b)
    wz = 2 * np.pi * (np.sign(d) if lo == abs(d) else d / lo) - 2 * np.pi * d / b if d != 0 else 0.0
    assert abs(o["W"][2] - wz) < 1e-12
    assert np.abs(o["W"][:2]).max() < 1e-10 * max(1.0, b * b)


def potential_closed_form(P, r):
    """int_T 1/R ds' for a flat triangle: the classical edge-sum formula
    (Wilton et al. 1984; Graglia 1993)."""
    n = np.cross(P[1] - P[0], P[2] - P[0])
    n /= np.linalg.norm(n)
    d = np.dot(r - P[0], n)
    p = r - d * n
    tot = 0.0
    for i in range(3):
        a, b = P[i], P[(i + 1) % 3]
        s = (b - a) / np.linalg.norm(b - a)
        m = np.cross(s, n)  # outward in-plane normal for a CCW triangle
        t0 = np.dot(a - p, m)
        lm, lp = np.dot(a - p, s), np.dot(b - p, s)
        Rm, Rp = np.linalg.norm(r - a), np.linalg.norm(r - b)
        R0sq = t0 * t0 + d * d
        tot += t0 * np.log((Rp + lp) / (Rm + lm))
        ad = abs(d)
        if ad > 0:
            tot -= ad * (np.arctan(t0 * lp / (R0sq + ad * Rp)) - np.arctan(t0 * lm / (R0sq + ad * Rm)))
    return tot


TRI = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.3, 0.8, 0.0]])


@pytest.mark.parametrize("r", [
    [0.4, 0.3, 0.0], [0.4, 0.3, 0.05], [1.5, 1.0, 0.2], [-0.3, 0.4, -0.1], [0.5, 0.05, 0.01],
])
def test_static_potential_matches_closed_form(r):
    r = np.array(r)
    for n_psi, tol in ((16, 1e-11), (10, 1e-6), (6, 1e-4)):
        o = Q.inner_moments(TRI, r, 0.0, np.inf, 0, 1.0, Q.Spec(n_psi=n_psi))
        ex = potential_closed_form(TRI, r)
        assert abs(o["I0"] - ex) < tol * abs(ex), (n_psi, o["I0"], ex)


def _brute(P, r, fun, level=6):
    """Subdivided 7-point product rule (for points away from the triangle)."""
    bary, w = Q.radon7()
    tris = [P]
    for _ in range(level):
        nt = []
        for T in tris:
            m01, m12, m20 = (T[0] + T[1]) / 2, (T[1] + T[2]) / 2, (T[2] + T[0]) / 2
            nt += [np.array([T[0], m01, m20]), np.array([m01, T[1], m12]),
                   np.array([m20, m12, T[2]]), np.array([m01, m12, m20])]
        tris = nt
    acc = 0.0
    for T in tris:
        A = 0.5 * np.linalg.norm(np.cross(T[1] - T[0], T[2] - T[0]))
        pts = bary @ T
        acc = acc + A * np.einsum("q,q...->...", w, fun(pts))
    return acc


def test_vector_moments_against_brute_force():
    P = np.array([[0.0, 0.0, 0.1], [1.0, 0.1, 0.0], [0.3, 0.8, 0.2]])
    r = np.array([0.9, 1.3, 0.7])
    spec = Q.Spec(n_psi=16)
    o = Q.inner_moments(P, r, 0.0, np.inf, 0, 1.0, spec)
    n = np.cross(P[1] - P[0], P[2] - P[0])
    n /= np.linalg.norm(n)
    p = r - np.dot(r - P[0], n) * n

    def Rof(x):
        return np.linalg.norm(r - x, axis=-1)

    I0 = _brute(P, r, lambda x: 1.0 / Rof(x), 4)
    Iu = _brute(P, r, lambda x: (x - p) / Rof(x)[:, None], 4)
    W = _brute(P, r, lambda x: (r - x) / Rof(x)[:, None] ** 3, 4)
    assert abs(o["I0"] - I0) < 1e-12
    assert np.abs(o["Iu"] - Iu).max() < 1e-12
    assert np.abs(o["W"] - W).max() < 1e-11


@pytest.mark.parametrize("r", [[0.4, 0.3, 0.03], [1.2, 0.9, 0.3], [0.5, -0.4, 0.0]])
def test_shells_partition_static(r):
    """Summing shell integrals over all shells reproduces the whole-triangle
    integral, although the angular break points differ."""
    r = np.array(r)
    spec = Q.Spec(n_psi=16)
    dt = 0.07
    st = Q.inner_moments(TRI, r, 0.0, np.inf, 0, 1.0, spec)
    acc = {"I0": 0.0, "Iu": np.zeros(3), "W": np.zeros(3)}
    for j in range(40):
        o = Q.inner_moments(TRI, r, j * dt, (j + 1) * dt, j, dt, spec)
        for k in acc:
            acc[k] = acc[k] + o[k]
    for k in acc:
        assert np.abs(np.asarray(acc[k]) - np.asarray(st[k])).max() < 1e-9 * (1 + np.abs(st[k]).max())


def test_angular_convergence():
    r = np.array([0.45, 0.32, 0.02])
    a = Q.inner_moments(TRI, r, 0.21, 0.28, 3, 0.07, Q.Spec(n_psi=8))
    b = Q.inner_moments(TRI, r, 0.21, 0.28, 3, 0.07, Q.Spec(n_psi=20))
    for k in ("I0", "Iu", "Sx", "W"):
        assert np.abs(np.asarray(a[k]) - np.asarray(b[k])).max() < 1e-7 * (1 + np.abs(b[k]).max())
