"""Temporal basis pairs of higher order in the oracle (Remark of Sec. IV-B;
the bases of Sec. IV-A; oracle/temporal.py).

Pins:
  * the basis: the shifted quadratic (p = 2) and the hat (p = 1) interpolators
    written out here from the Lagrange formula; partition of unity and
    reproduction of polynomials up to degree p; q_0' = (h_0 - h_1)/dt at
    points off the nodes; q_0 = the integral of h_0 - h_1 (adaptive
    quadrature of the definition); q_0 of compact support [-dt, (p+1) dt);
  * the lag combinations: for random lags and distances the x-polynomial of
    the interval equals q_0, h_0' and h_0 + R h_0' at the retarded time;
  * p = 1 through the general combinations equals the closed forms of the
    hat functions (A, B, C on the tetrahedron, to rounding);
  * the x-weighted shell moments V^(1), S^(3), N^(1), N^(2) against the
    independent integrator (tests/brute_quadrature.py) with weights x^a;
  * the march with p = 2: late-time decay, and a smaller time-discretisation
    error than p = 1 at the same time step against a 4x finer p = 1 march."""
import math

import numpy as np
import pytest
from scipy import integrate

import brute_quadrature as BQ

TOL = 1e-11  # x-moment entries against the brute integrator (48 angular points)


def lagrange_h0(p, u):
    """h_0 at u = t/dt from the definition: on [m-1, m) the Lagrange
    polynomial through the nodes m-p..m that is 1 at 0."""
    if u < -1.0 or u >= p:
        return 0.0
    m = math.floor(u) + 1
    val = 1.0
    for n in range(m - p, m + 1):
        if n != 0:
            val *= (u - n) / (0.0 - n)
    return val


def q0_by_quadrature(p, u):
    if u <= -1.0:
        return 0.0
    pts = [float(v) for v in range(0, int(math.floor(u)) + 1) if -1.0 < v < u]
    val, _ = integrate.quad(lambda v: lagrange_h0(p, v) - lagrange_h0(p, v - 1.0), -1.0, u, points=pts or None,
                            epsabs=1e-14, epsrel=1e-13, limit=200)
    return val


@pytest.mark.parametrize("p", [1, 2])
def test_basis_against_the_definition(p):
    from oracle import temporal as T
    rng = np.random.default_rng(p)
    for u in rng.uniform(-1.5, p + 1.5, 400):
        assert abs(T.h0(p, u) - lagrange_h0(p, u)) < 1e-14
    for u in np.linspace(-0.97, 6.93, 157):
        for r in range(p + 1):
            tot = sum((i ** r) * T.h0(p, u - i) for i in range(-3, 12))
            assert abs(tot - u ** r) < 1e-11 * max(1.0, abs(u) ** r)


@pytest.mark.parametrize("p", [1, 2])
def test_q0_identity_and_support(p):
    from oracle import temporal as T
    eps = 1e-6
    for u in np.linspace(-0.9, p + 0.9, 61):
        if abs(u - round(u)) < 1e-3:
            continue
        dq = (T.q0(p, u + eps) - T.q0(p, u - eps)) / (2 * eps)
        assert abs(dq - (lagrange_h0(p, u) - lagrange_h0(p, u - 1.0))) < 1e-7
        assert abs(T.q0(p, u) - q0_by_quadrature(p, u)) < 1e-12
    assert T.q0(p, -1.0) == 0.0 and abs(T.q0(p, p + 1.0)) < 1e-14 and abs(T.q0(p, p + 3.0)) < 1e-14
    for n in range(0, p + 2):  # continuous at the nodes
        assert abs(T.q0(p, n - 1e-12) - T.q0(p, n)) < 1e-10


@pytest.mark.parametrize("p", [1, 2])
def test_combinations_against_the_basis(p):
    from oracle import temporal as T
    da, qa, ca = T.combos(p)
    rng = np.random.default_rng(10 + p)
    for _ in range(300):
        k = int(rng.integers(0, 14))
        Rn = float(rng.uniform(1e-3, k + p + 1.9))
        if abs(Rn - round(Rn)) < 1e-4 or abs((k - Rn) - round(k - Rn)) < 1e-4:
            continue
        j = math.ceil(Rn) - 1
        x, m, u = Rn - j, k - j, k - Rn
        got_q = sum(qa[m][a] * x ** a for a in range(p + 2)) if 0 <= m <= p + 1 else 0.0
        assert abs(got_q - q0_by_quadrature(p, u)) < 1e-11
        e = 1e-6
        dh = (lagrange_h0(p, u + e) - lagrange_h0(p, u - e)) / (2 * e)
        got_d = sum(da[m][a] * x ** a for a in range(p)) if 0 <= m <= p else 0.0
        assert abs(got_d - dh) < 1e-7
        got_c = sum(ca(k, m)[a] * x ** a for a in range(p + 1)) if 0 <= m <= p else 0.0
        assert abs(got_c - (lagrange_h0(p, u) + Rn * dh)) < 1e-6 * max(1.0, Rn)


def test_order1_general_equals_the_hat_closed_forms():
    from oracle import operators as O
    from test_oracle_entries import tetrahedron
    xyz, tri = tetrahedron()
    asm = O.Assembly(xyz, tri, 0.4)
    G = asm.gram()
    V, S, N = asm.shells()
    A1, B1, C1 = asm.lag_matrices(V, S, N, G)
    A2, B2, C2 = asm.lag_matrices_order(V, S, N, G, order=1)
    for X1, X2 in ((A1, A2), (B1, B2), (C1, C2)):
        scale = max(np.abs(x).max() for x in X1)
        assert max(np.abs(a - b).max() for a, b in zip(X1, X2)) < 1e-14 * scale


@pytest.fixture(scope="module")
def order2_tetra():
    from oracle import operators as O, quadrature as Q
    from test_oracle_entries import tetrahedron
    xyz, tri = tetrahedron()
    dt = 0.4
    asm = O.Assembly(xyz, tri, dt, spec=Q.Spec(n_psi=48), order=2)
    V, S, N = asm.shells()
    return dict(asm=asm, V=V, S=S, N=N, mesh=BQ.Mesh(asm.topo), dt=dt)


def test_x_moments_against_the_brute_integrator(order2_tetra):
    """V^(1), S^(3), N^(1), N^(2) entries (x = R/dt - j) on every shell, for an
    edge with itself, with an edge of a shared triangle and with a vertex
    neighbour; a triangle with itself and with a neighbour."""
    from test_oracle_entries import _edge_pairs, _tri_pairs
    c = order2_tetra
    asm, V, S, N, mesh, dt = c["asm"], c["V"], c["S"], c["N"], c["mesh"], c["dt"]
    assert V.shape[1] == 2 and S.shape[1] == 4 and N.shape[1] == 3
    worst = {"V1": 0.0, "S3": 0.0, "N1": 0.0, "N2": 0.0}
    pairs = _edge_pairs(asm.topo)[:3]
    for j in range(V.shape[0]):
        lo, hi = j * dt, (j + 1) * dt
        sv = np.abs(V[j, 1]).max()
        for m, n in pairs:
            if sv > 0.0:
                b = 0.5 * (BQ.v_shell(mesh, m, n, lo, hi, dt=dt, xa=1) + BQ.v_shell(mesh, n, m, lo, hi, dt=dt, xa=1))
                worst["V1"] = max(worst["V1"], abs(V[j, 1, m, n] - b) / sv)
            for a in (1, 2):
                sn = np.abs(N[j, a]).max()
                if sn > 0.0:
                    worst["N%d" % a] = max(worst["N%d" % a],
                                           abs(N[j, a, m, n] - BQ.n_shell(mesh, m, n, lo, hi, dt=dt, xa=a)) / sn)
        ss = np.abs(S[j, 3]).max()
        if ss > 0.0:
            for cc, cs in _tri_pairs(asm.topo)[:2]:
                b = 0.5 * (BQ.s_shell(mesh, cc, cs, j, dt)[3] + BQ.s_shell(mesh, cs, cc, j, dt)[3])
                worst["S3"] = max(worst["S3"], abs(S[j, 3, cc, cs] - b) / ss)
    print("[tetrahedron, p = 2] x-moment entries: worst %s of the largest entry" % worst)
    assert max(worst.values()) < TOL


def test_order2_march_is_stable_and_more_accurate():
    """120-edge sphere, c dt = 0.15 m, a modulated Gaussian at 0.5 per metre
    (about 13 steps a period), 160 m of time: both orders decay to below
    1e-15 of the peak; against p = 1 at dt/4 the p = 2 march is closer than
    the p = 1 march at the same dt (measured 2.8e-2 against 4.0e-2)."""
    from oracle import operators as O, excitation as E, mot
    from workloads import meshes, waves
    xyz, tri = meshes.icosphere(1)
    f0, dt, t_end = 0.5, 0.15, 160.0
    res = {}
    for order, d in ((1, dt / 4), (1, dt), (2, dt)):
        asm = O.Assembly(xyz, tri, d, order=order)
        asm.build()
        assert asm.K == O.n_lags(asm.D, d, order)
        w = waves.Wave((0.0, 0.0, -1.0), (1.0, 0.0, 0.0), 1.0, waves.mod_gauss_t0(f0, asm.D), 0, 0.0, f0, f0)
        n = int(round(t_end / d))
        j = mot.currents(asm.proj.PLH, asm.proj.PS, asm.dtn, mot.march(asm.T, E.rhs(asm, w, n)))
        nrm = np.linalg.norm(j, axis=1)
        assert nrm[len(nrm) // 2:].max() < 1e-15 * nrm.max()
        res[(order, d)] = j
    ref = res[(1, dt / 4)][3::4]
    err = {}
    for order in (1, 2):
        j = res[(order, dt)]
        m = min(len(j), len(ref))
        err[order] = np.linalg.norm(j[:m] - ref[:m], axis=1).max() / np.linalg.norm(ref, axis=1).max()
    print("[sphere120] error against p = 1 at dt/4: p = 1 %.3e, p = 2 %.3e" % (err[1], err[2]))
    assert err[2] < 0.8 * err[1]
