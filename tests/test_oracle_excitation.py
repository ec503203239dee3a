"""Pins of the oracle's tested incident field (Sec. II-C): the RWG-tested
electric field e_m(t) = integral of f_m . e_in over the two cells of edge m,
against adaptive integration with the RWG function written from its
definition (unit flux through the edge, pointing away from the free vertex
on the plus cell and towards it on the minus cell)."""
import numpy as np
from scipy import integrate

from oracle import excitation as E
from oracle import operators as O
from workloads import meshes, waves


def _gaussian(t, wave, r):
    """The paper's Gaussian plane wave (Sec. V), e = g(t - t0 - k.r) p."""
    u = t - wave.t0 - r @ np.asarray(wave.k_hat)
    return 4.0 * wave.amplitude / (wave.w * np.sqrt(np.pi)) * np.exp(-((4.0 / wave.w) * u) ** 2) * np.asarray(wave.pol)


def _tested_brute(topo, m, wave, t):
    total = 0.0
    for side, c in ((1.0, topo.cells[m, 0]), (-1.0, topo.cells[m, 1])):
        P = topo.xyz[topo.tri[c]]
        free = [v for v in topo.tri[c] if v not in topo.edges[m]]
        assert len(free) == 1
        pf = topo.xyz[free[0]]
        area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))

        def integrand(v, u):
            r = P[0] + u * (P[1] - P[0]) + v * (P[2] - P[0])
            f = side * (r - pf) / (2.0 * area)
            return float(f @ _gaussian(t, wave, r)) * 2.0 * area

        val, _ = integrate.dblquad(integrand, 0.0, 1.0, 0.0, lambda u: 1.0 - u, epsabs=1e-14, epsrel=1e-12)
        total += val
    return total


def test_tested_electric_field_against_adaptive_integration():
    xyz, tri = meshes.icosphere(1)
    dt = 0.15
    a = O.Assembly(xyz, tri, dt)
    kh = (0.3, -0.4, np.sqrt(0.75))
    ph = tuple(np.array([0.0, np.sqrt(0.75), 0.4]) / np.sqrt(0.91))  # k x (1, 0, 0), normalised
    wave = waves.Wave(kh, ph, 1.0, 3.0, 1, 6.0, 0.0, 0.0)
    k, p = np.asarray(wave.k_hat), np.asarray(wave.pol)
    assert abs(np.linalg.norm(k) - 1) < 1e-12 and abs(np.linalg.norm(p) - 1) < 1e-12 and abs(k @ p) < 1e-12
    n = 30
    e, _ = E.tested_fields(a, wave, n)
    step = int(np.argmax(np.abs(e).max(axis=1)))  # the pulse on the sphere
    t = (step + 1) * dt
    scale = np.abs(e[step]).max()
    for m in (0, 7, 33, 64, 101, a.topo.ne - 1):
        ref = _tested_brute(a.topo, m, wave, t)
        assert abs(e[step, m] - ref) < 1e-7 * scale, (m, e[step, m], ref)


def test_testing_maps_integrate_a_uniform_field_exactly():
    """For a uniform field F and a divergence-conforming function g with no
    flux out of its support, the integral of g . F over the surface is
    -F . (integral of r div g) (divergence theorem cell by cell, with the
    normal flux continuous across inner edges).  Unit-flux RWG functions:
    div f_m = +1/A on the plus cell and -1/A on the minus cell, so
    integral f_m = centroid(minus) - centroid(plus).  BC functions on the
    barycentric refinement: div g = (sum of the fine-cell fluxes) / A on
    each fine cell.  The oracle's testing maps (7-point rule, exact for the
    linear integrands here) must agree to rounding."""
    xyz, tri = meshes.torus(1.0, 0.4, 12, 6)
    a = O.Assembly(xyz, tri, 0.12)
    t = a.topo
    We, pc, Wh, pf = E._testing_matrices(a)
    F = np.array([0.3, -1.1, 0.7])
    e = We @ np.tile(F, pc.shape[0])
    h = Wh @ np.tile(F, pf.shape[0])
    int_f = t.centroid[t.cells[:, 1]] - t.centroid[t.cells[:, 0]]
    assert np.abs(e - int_f @ F).max() < 1e-13 * np.abs(e).max()
    fc = t.fxyz[t.ftri].mean(axis=1)
    int_g = np.zeros((t.ne, 3))
    for ft, lst in enumerate(t.bc_entries):
        for m, fl in lst:
            int_g[m] -= float(np.sum(fl)) * fc[ft]
    assert np.abs(h - int_g @ F).max() < 1e-12 * np.abs(h).max()
