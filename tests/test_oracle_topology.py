"""Pins of the oracle's mesh topology, RWG and BC bases (Sec. II-C, II-D)."""
import numpy as np
import pytest

from oracle.topology import Topology, MeshError, field_at
from workloads import meshes


@pytest.mark.parametrize("maker,counts,genus", [
    (lambda: meshes.icosphere(2), (162, 480, 320), 0),
    (lambda: meshes.icosphere(4), (2562, 7680, 5120), 0),
    (lambda: meshes.torus(1.0, 0.3, 80, 25), (2000, 6000, 4000), 1),
    (lambda: meshes.cube(1.5, 3), (56, 162, 108), 0),
    (lambda: meshes.tetrahedron(), (4, 6, 4), 0),
])
def test_mesh_counts_euler_orientation(maker, counts, genus):
    xyz, tri = maker()
    t = Topology(xyz, tri) if counts[1] < 3000 else None
    assert (len(xyz), len(tri)) == (counts[0], counts[2])
    assert counts[0] - counts[1] + counts[2] == 2 - 2 * genus
    assert meshes.outward_volume(xyz, tri) > 0
    if t is not None:
        assert t.ne == counts[1]
        assert t.n_harmonic == 2 * genus


def test_incidence_identities():
    for xyz, tri in [meshes.icosphere(1), meshes.torus(1.0, 0.4, 8, 5)]:
        t = Topology(xyz, tri)
        L, S = t.Lambda.toarray(), t.Sigma.toarray()
        assert np.all(L @ np.ones(t.nv) == 0)
        assert np.all(S @ np.ones(t.nc) == 0)
        assert np.all(S.T @ L == 0)  # loops are divergence free (exact integers)
        # harmonic dimension: kernel of [Lambda Sigma]^T has dim N_H (Sec. II-D)
        M = np.concatenate([L, S], axis=1)
        nullity = t.ne - np.linalg.matrix_rank(M)
        assert nullity == t.n_harmonic


def test_mesh_validation():
    xyz, tri = meshes.icosphere(1)
    with pytest.raises(MeshError):
        Topology(xyz, tri[:-1])  # open surface
    bad = tri.copy()
    bad[0] = bad[0][::-1]
    with pytest.raises(MeshError):
        Topology(xyz, bad)  # inconsistent orientation


def _edge_flux(P, A, fl, i):
    """Outward flux of the RT0 field through the edge opposite vertex i,
    integrated with the 2-point Gauss rule (exact for linear normal data)."""
    a, b = P[(i + 1) % 3], P[(i + 2) % 3]
    n = np.cross(P[1] - P[0], P[2] - P[0])
    n /= np.linalg.norm(n)
    t = b - a
    nu = np.cross(t, n)
    nu /= np.linalg.norm(nu)
    L = np.linalg.norm(t)
    g = 0.5 / np.sqrt(3.0)
    pts = np.array([a + (0.5 - g) * t, a + (0.5 + g) * t])
    v = field_at(P, A, fl, pts)
    return L * 0.5 * np.sum(v @ nu)


def test_rwg_unit_flux_and_divergence():
    xyz, tri = meshes.icosphere(1)
    t = Topology(xyz, tri)
    for c in range(t.nc):
        P = t.xyz[t.tri[c]]
        for i in range(3):
            fl = np.zeros(3)
            fl[i] = t.tri_sign[c, i]
            m = t.tri_edge[c, i]
            # f_m flows out of c+ with unit flux (Sec. II-C, no length factor)
            expect = 1.0 if t.cells[m, 0] == c else -1.0
            assert abs(_edge_flux(P, t.area[c], fl, i) - expect) < 1e-13
            # the r+ of the printed definition is the vertex opposite e_m
            assert set(t.tri[c]) - set(t.edges[m]) == {t.tri[c, i]}


def test_bc_flux_charge_and_continuity():
    for xyz, tri in [meshes.icosphere(1), meshes.torus(1.0, 0.4, 8, 5)]:
        t = Topology(xyz, tri)
        # per fine edge, outward fluxes seen from both sides cancel (div-conforming)
        fedge = {}
        for ft in range(6 * t.nc):
            v = t.ftri[ft]
            for i in range(3):
                key = tuple(sorted((v[(i + 1) % 3], v[(i + 2) % 3])))
                fedge.setdefault(key, []).append((ft, i))
        per = {}
        for ft, lst in enumerate(t.bc_entries):
            for e, fl in lst:
                per.setdefault(e, {})[ft] = fl
        for m in range(t.ne):
            fm = per[m]
            for key, uses in fedge.items():
                assert len(uses) == 2
                (t1, i1), (t2, i2) = uses
                f1 = fm[t1][i1] if t1 in fm else 0.0
                f2 = fm[t2][i2] if t2 in fm else 0.0
                assert abs(f1 + f2) < 1e-14
            # divergence: -Lambda_mv / (2 N_v A_t) on the dual cell of v
            vm, vp = t.edges[m]
            for ft, fl in fm.items():
                v = t.fowner[ft]
                lam = 1.0 if v == vp else (-1.0 if v == vm else 0.0)
                assert lam != 0.0
                assert abs(fl.sum() - (-lam / (2.0 * t.valence[v]))) < 1e-14
            # unit flux across the dual edge: fine edges (m_e, g_c+-)
            mid = t.nv + m
            tot = 0.0
            for ft, fl in fm.items():
                if t.fowner[ft] != vm:
                    continue
                vv = t.ftri[ft]
                if mid in vv:
                    tot += fl[0]  # edge opposite the coarse vertex
            assert abs(tot - 1.0) < 1e-14
        # BC loops: sum_m Sigma_mc g_m is divergence free on every fine triangle
        S = t.Sigma.toarray()
        for c in range(0, t.nc, 7):
            div = np.zeros(6 * t.nc)
            for ft, lst in enumerate(t.bc_entries):
                for e, fl in lst:
                    div[ft] += S[e, c] * fl.sum()
            assert np.abs(div).max() < 1e-14


def test_gram_well_conditioned_under_refinement():
    from oracle.operators import Assembly
    conds = []
    for s in (1, 2, 3):
        xyz, tri = meshes.icosphere(s)
        asm = Assembly(xyz, tri, 0.1, K=1)
        conds.append(np.linalg.cond(asm.gram()))
    # BC functions are the dual of RWGs: the Gram stays well-conditioned
    assert max(conds) < 5.0
    assert conds[-1] < 1.2 * conds[0] + 1.0
