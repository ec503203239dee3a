"""Single entries of the oracle's assembled matrices against integrals
written from their definitions (tests/brute_quadrature.py), on the
tetrahedron and the icosahedron, and on a tetrahedron a hundred times
smaller than the time step (the small-argument forms of the Yukawa
remainders).

The quadrature specification fixes the test (outer) rules; the source
(inner) integrals are computed here by another method than the oracle's
(Duffy fans from the closest point with the shell limits solved on every
ray, graded Gauss-Legendre; basis fields built from their fluxes), so a
mistake in the oracle's polar scheme, shell ranges, projection-point terms,
basis evaluations or accumulation shows as a disagreement.

Covered (Sec. II-A, II-C, IV-A): the retarded shell moments V_j (RWG-RWG),
S_j^p (triangle-triangle) and N_j (BC-RWG) for self, edge-sharing,
vertex-sharing and separated pairs on every shell they reach, and the
static Yukawa operators Z^s, Z^h and M.  The oracle is assembled with 48
angular Gauss points per sub-interval, where its scheme is converged: the
entries agree to 1e-11 of the largest entry of the matrix compared.  With
the 10 points the library and the oracle both use for the workloads, the
angular rule's own error shows: within 1e-7 (measured 1.8e-8, on the
shells that contain the singular self pairs)."""
import numpy as np
import pytest

import brute_quadrature as BQ

TOL = 1e-11       # oracle with 48 angular points
TOL_SPEC = 1e-7   # oracle with the 10 angular points of the workloads


def tetrahedron():
    """Regular tetrahedron inscribed in the unit sphere, faces counter-clockwise
    seen from outside."""
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64) / np.sqrt(3.0)
    faces = []
    for f in ([0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]):
        p = v[f]
        n = np.cross(p[1] - p[0], p[2] - p[0])
        faces.append(f if np.dot(n, p.mean(axis=0)) > 0 else [f[0], f[2], f[1]])
    return v, np.array(faces, dtype=np.int32)


@pytest.fixture(scope="module", params=["tetrahedron", "icosahedron", "small tetrahedron"])
def case(request):
    from oracle import operators as O
    from workloads import meshes
    if request.param == "tetrahedron":
        xyz, tri = tetrahedron()
        dt = 0.4
    elif request.param == "small tetrahedron":
        # edge 0.016 m against c dt = 1 m: kappa R < 0.02 on every pair, where
        # the Yukawa remainders take their small-argument forms
        xyz, tri = tetrahedron()
        xyz = 0.01 * xyz
        dt = 1.0
    else:
        xyz, tri = meshes.icosphere(0)
        dt = 0.3
    from oracle import quadrature as Q
    asm = O.Assembly(xyz, tri, dt, spec=Q.Spec(n_psi=48))
    V, S, N = asm.shells()
    V10 = O.Assembly(xyz, tri, dt).shells()[0]
    return dict(name=request.param, asm=asm, V=V, V10=V10, S=S, N=N, mesh=BQ.Mesh(asm.topo), dt=dt)


def _edge_pairs(t):
    """An edge with itself, with an edge of a shared triangle, with an edge
    sharing only a vertex, and with an edge sharing nothing (if any)."""
    m = 0
    tris_m = set(t.cells[m])
    verts_m = set(t.edges[m])
    same_tri = next(n for n in range(t.ne) if n != m and set(t.cells[n]) & tris_m)
    vert_only = [n for n in range(t.ne) if not (set(t.cells[n]) & tris_m) and set(t.edges[n]) & verts_m]
    far = [n for n in range(t.ne) if not set(t.edges[n]) & verts_m and not (set(t.cells[n]) & tris_m)]
    out = [(m, m), (m, same_tri)]
    if vert_only:
        out.append((m, vert_only[0]))
    if far:
        out.append((m, far[len(far) // 2]))
    return out


def _tri_pairs(t):
    """A triangle with itself, an edge neighbour, a vertex neighbour and a
    separated triangle (those that exist)."""
    c = 0
    vc = set(t.tri[c])
    out = [(c, c)]
    edge_nb = [d for d in range(t.nc) if d != c and len(vc & set(t.tri[d])) == 2]
    vert_nb = [d for d in range(t.nc) if len(vc & set(t.tri[d])) == 1]
    far = [d for d in range(t.nc) if not vc & set(t.tri[d])]
    for lst in (edge_nb, vert_nb, far):
        if lst:
            out.append((c, lst[-1]))
    return out


def test_vector_potential_shells(case):
    """V_j[m][n] = int int_{j dt < R <= (j+1) dt} f_m . f_n / (4 pi R)
    (symmetrised as the oracle does), every shell."""
    asm, V, V10, mesh, dt = case["asm"], case["V"], case["V10"], case["mesh"], case["dt"]
    worst = worst10 = 0.0
    for m, n in _edge_pairs(asm.topo):
        for j in range(V.shape[0]):
            b = 0.5 * (BQ.v_shell(mesh, m, n, j * dt, (j + 1) * dt) + BQ.v_shell(mesh, n, m, j * dt, (j + 1) * dt))
            scale = np.abs(V[j]).max()
            if scale == 0.0:
                assert b == 0.0
                continue
            worst = max(worst, abs(V[j, m, n] - b) / scale)
            worst10 = max(worst10, abs(V10[j, m, n] - b) / scale)
    print("[%s] V_j entries: worst %.2e of the largest entry (%.2e with 10 angular points)"
          % (case["name"], worst, worst10))
    assert worst < TOL and worst10 < TOL_SPEC


def test_scalar_potential_moments(case):
    """S_j^p[c][c'] = int_c int_{c', shell j} x^p / (4 pi R), x = R/dt - j,
    p = 0, 1, 2 (symmetrised), every shell."""
    asm, S, mesh, dt = case["asm"], case["S"], case["mesh"], case["dt"]
    worst = 0.0
    for c, cs in _tri_pairs(asm.topo):
        for j in range(S.shape[0]):
            b = 0.5 * (BQ.s_shell(mesh, c, cs, j, dt) + BQ.s_shell(mesh, cs, c, j, dt))
            for p in range(3):
                scale = np.abs(S[j, p]).max()
                if scale > 0.0:
                    worst = max(worst, abs(S[j, p, c, cs] - b[p]) / scale)
    print("[%s] S_j^p entries: worst %.2e of the largest entry" % (case["name"], worst))
    assert worst < TOL


def test_mfie_shells(case):
    """N_j[m][n] = int int_{shell j} g_m . ((r - r') x f_n) / (4 pi R^3), BC
    test against RWG trial, every shell."""
    asm, N, mesh, dt = case["asm"], case["N"], case["mesh"], case["dt"]
    worst = 0.0
    for m, n in _edge_pairs(asm.topo):
        for j in range(N.shape[0]):
            b = BQ.n_shell(mesh, m, n, j * dt, (j + 1) * dt)
            scale = np.abs(N[j]).max()
            if scale > 0.0:
                worst = max(worst, abs(N[j, m, n] - b) / scale)
    print("[%s] N_j entries: worst %.2e of the largest entry" % (case["name"], worst))
    assert worst < TOL


def test_static_yukawa_entries(case):
    """Z^s = -kappa int int g.g G_kappa, Z^h = -(1/kappa) int int div g div g
    G_kappa (through the dual-cell sums; div g_m = -Lambda_mv/(2 N_v A_t) on
    the fine triangles of the dual cell of v) and M = int int
    g.((r - r') x f)(1 + kappa R) e^{-kappa R}/(4 pi R^3), kappa = 1/dt."""
    asm, mesh = case["asm"], case["mesh"]
    t = asm.topo
    kappa = asm.kappa
    Zs, Zh, M = asm.yukawa()  # the assembly's own angular rule (48 points here)
    Lam = t.Lambda.toarray()
    worst = {"Zs": 0.0, "Zh": 0.0, "M": 0.0}
    for m, n in _edge_pairs(t):
        b = -kappa * 0.5 * (BQ.yukawa_bc_pair(mesh, m, n, kappa) + BQ.yukawa_bc_pair(mesh, n, m, kappa))
        worst["Zs"] = max(worst["Zs"], abs(Zs[m, n] - b) / np.abs(Zs).max())
        zh = 0.0
        for v in t.edges[m]:
            for vs in t.edges[n]:
                d = 0.5 * (BQ.yukawa_dual_pair(mesh, v, vs, kappa) + BQ.yukawa_dual_pair(mesh, vs, v, kappa))
                zh += (Lam[m, v] / (2.0 * t.valence[v])) * d * (Lam[n, vs] / (2.0 * t.valence[vs]))
        zh *= -1.0 / kappa
        worst["Zh"] = max(worst["Zh"], abs(Zh[m, n] - zh) / np.abs(Zh).max())
        b = BQ.mfie_pair(mesh, m, n, kappa)
        worst["M"] = max(worst["M"], abs(M[m, n] - b) / np.abs(M).max())
    print("[%s] Yukawa entries: worst %s of the largest entry" % (case["name"], worst))
    assert max(worst.values()) < TOL
