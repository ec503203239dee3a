"""Mesh topology, RWG and Buffa-Christiansen bases (oracle; test infrastructure).

Follows Sec. II-C (RWG definition with no edge-length factor, BC functions on
the barycentric refinement) and Sec. II-D (vertex-edge matrix Lambda and
face-edge matrix Sigma).

Readings of the paper used here (the paper does not state them):
  * Edge numbering: edges sorted by (min vertex, max vertex), oriented
    v- = min -> v+ = max.  The paper only says an edge is oriented from v- to
    v+.
  * c+ of an edge is the triangle whose counter-clockwise vertex cycle
    traverses v- -> v+; c- is the other one.  Any rule used uniformly makes
    Sigma^T Lambda = 0; this one is fixed so both implementations agree.
  * RWG f_n is (r - r+)/(2A+) on c+ and (r- - r)/(2A-) on c-, i.e. outward
    flux +1 through e_n from c+ (the unit-flux form printed in Sec. II-C).
  * BC coefficients (cited, not printed, in the paper): built from unit-flux
    RWGs on the barycentric refinement so that flux 1/2 crosses each of the
    two fine edges of the dual edge of e_n (from the dual cell of v- into the
    dual cell of v+), and the charge +-1 is spread equally, 1/(2N_v) per fine
    triangle, over the 2N_v fine triangles of each dual cell.  This makes the
    BC divergence factor through Lambda^T, which the projector identity
    P^{Sigma H} Z^h = 0 of Sec. III-B requires.

Every divergence-conforming field on a triangle with vertices P0, P1, P2 and
area A is stored as its three outward fluxes (F0, F1, F2) through the edges
opposite P0, P1, P2:  v(r) = sum_i F_i (r - P_i) / (2A).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class MeshError(ValueError):
    pass


class Topology:
    def __init__(self, xyz, tri):
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int64)
        self.nv = self.xyz.shape[0]
        self.nc = self.tri.shape[0]
        self._edges()
        self._geometry()
        self._refine()
        self._bc()

    # ---------------------------------------------------------------- edges
    def _edges(self):
        tri = self.tri
        edict: dict[tuple[int, int], list] = {}
        for c in range(self.nc):
            for i in range(3):
                a, b = int(tri[c, (i + 1) % 3]), int(tri[c, (i + 2) % 3])
                key = (min(a, b), max(a, b))
                edict.setdefault(key, []).append((c, i, a, b))
        keys = sorted(edict)
        ne = len(keys)
        edges = np.zeros((ne, 2), dtype=np.int64)
        cells = np.full((ne, 2), -1, dtype=np.int64)
        tri_edge = np.zeros((self.nc, 3), dtype=np.int64)
        tri_sign = np.zeros((self.nc, 3), dtype=np.int64)
        for m, key in enumerate(keys):
            uses = edict[key]
            if len(uses) != 2:
                raise MeshError("edge %s used by %d triangles (open or non-manifold)" % (key, len(uses)))
            edges[m] = key
            plus = [u for u in uses if u[2] == key[0]]  # traverses v- -> v+
            minus = [u for u in uses if u[2] == key[1]]
            if len(plus) != 1 or len(minus) != 1:
                raise MeshError("edge %s inconsistently oriented" % (key,))
            cells[m, 0] = plus[0][0]
            cells[m, 1] = minus[0][0]
            tri_edge[plus[0][0], plus[0][1]] = m
            tri_sign[plus[0][0], plus[0][1]] = 1
            tri_edge[minus[0][0], minus[0][1]] = m
            tri_sign[minus[0][0], minus[0][1]] = -1
        self.ne = ne
        self.edges = edges
        self.cells = cells
        self.tri_edge = tri_edge
        self.tri_sign = tri_sign
        # connectivity check (the paper assumes a connected surface)
        adj = sp.coo_matrix((np.ones(ne), (cells[:, 0], cells[:, 1])), shape=(self.nc, self.nc))
        ncomp, _ = sp.csgraph.connected_components(adj, directed=False)
        if ncomp != 1:
            raise MeshError("surface is not connected")
        self.euler = self.nv - self.ne + self.nc
        self.n_harmonic = 2 - self.euler  # N_H = 2*genus for a closed surface
        rows = np.repeat(np.arange(ne), 2)
        self.Lambda = sp.csr_matrix(
            (np.tile([-1.0, 1.0], ne), (rows, edges.reshape(-1))), shape=(ne, self.nv))
        self.Sigma = sp.csr_matrix(
            (np.tile([1.0, -1.0], ne), (rows, cells.reshape(-1))), shape=(ne, self.nc))

    def _geometry(self):
        p = self.xyz[self.tri]
        cr = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
        nrm = np.linalg.norm(cr, axis=1)
        if np.any(nrm <= 0):
            raise MeshError("zero-area triangle")
        self.area = 0.5 * nrm
        self.normal = cr / nrm[:, None]
        self.centroid = p.mean(axis=1)
        d = self.xyz[:, None, :] - self.xyz[None, :, :]
        self.diameter = float(np.sqrt((d * d).sum(-1)).max())

    # ------------------------------------------------- barycentric refinement
    def _refine(self):
        nv, ne, nc = self.nv, self.ne, self.nc
        mids = 0.5 * (self.xyz[self.edges[:, 0]] + self.xyz[self.edges[:, 1]])
        self.fxyz = np.concatenate([self.xyz, mids, self.centroid], axis=0)
        ftri = np.zeros((6 * nc, 3), dtype=np.int64)
        for c in range(nc):
            g = nv + ne + c
            for i in range(3):
                vi = self.tri[c, i]
                m_next = nv + self.tri_edge[c, (i + 2) % 3]  # edge {v_i, v_{i+1}}
                m_prev = nv + self.tri_edge[c, (i + 1) % 3]  # edge {v_{i-1}, v_i}
                ftri[6 * c + 2 * i] = (vi, m_next, g)
                ftri[6 * c + 2 * i + 1] = (vi, g, m_prev)
        self.ftri = ftri
        self.fparent = np.repeat(np.arange(nc), 6)
        self.fowner = ftri[:, 0].copy()  # coarse vertex whose dual cell holds it
        p = self.fxyz[ftri]
        cr = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
        self.farea = 0.5 * np.linalg.norm(cr, axis=1)
        self.fnormal = cr / (2.0 * self.farea[:, None])

    # ------------------------------------------------------------ BC basis
    def _bc(self):
        nv, ne = self.nv, self.ne
        # incident triangles of each vertex with the local index of the vertex
        inc: list[list[tuple[int, int]]] = [[] for _ in range(nv)]
        for c in range(self.nc):
            for i in range(3):
                inc[self.tri[c, i]].append((c, i))
        entries: list[list[tuple[int, np.ndarray]]] = [[] for _ in range(6 * self.nc)]
        self.valence = np.array([len(x) for x in inc], dtype=np.int64)
        for v in range(nv):
            tris = {c: i for c, i in inc[v]}
            n_v = len(tris)
            # walk counter-clockwise around v: radial r_{2j} = (v, midpoint of
            # {v, a}), fine tri (v, m_va, g_c), radial r_{2j+1} = (v, g_c),
            # fine tri (v, g_c, m_vb), then into the triangle holding v -> b
            c0 = inc[v][0][0]
            ring_tris: list[int] = []
            ring_mid_edge: list[int] = []
            c = c0
            for _ in range(n_v):
                i = tris[c]
                a, b = self.tri[c, (i + 1) % 3], self.tri[c, (i + 2) % 3]
                ring_mid_edge.append(self.tri_edge[c, (i + 2) % 3])  # {v, a}
                ring_tris += [6 * c + 2 * i, 6 * c + 2 * i + 1]
                nxt = None
                for cc, ii in inc[v]:
                    if self.tri[cc, (ii + 1) % 3] == b:
                        nxt = cc
                        break
                if nxt is None:
                    raise MeshError("vertex %d: broken fan" % v)
                c = nxt
            if c != c0 or len(set(ring_tris)) != 2 * n_v:
                raise MeshError("vertex %d: fan is not a single disc" % v)
            two_n = 2 * n_v
            for jm, e in enumerate(ring_mid_edge):
                s = 1.0 if self.edges[e, 1] == v else -1.0  # v+ is the sink
                i0 = 2 * jm
                F = [0.0] + [(n_v - j) / (2.0 * n_v) for j in range(1, two_n)] + [0.0]
                for j in range(1, two_n + 1):
                    t = ring_tris[(i0 + j - 1) % two_n]
                    fl = np.array([
                        -0.5 if j in (1, two_n) else 0.0,
                        F[j],
                        -F[j - 1],
                    ]) * s
                    entries[t].append((int(e), fl))
        self.bc_entries = entries

    # ------------------------------------------------------------- helpers
    def rwg_entries(self):
        """Per coarse triangle: list of (edge index, outward fluxes)."""
        out = []
        for c in range(self.nc):
            lst = []
            for i in range(3):
                fl = np.zeros(3)
                fl[i] = float(self.tri_sign[c, i])
                lst.append((int(self.tri_edge[c, i]), fl))
            out.append(lst)
        return out

    def bc_matrix_on_fine(self):
        """Dense-free description as arrays: (fine tri, edge, F0, F1, F2)."""
        rows = []
        for t, lst in enumerate(self.bc_entries):
            for e, fl in lst:
                rows.append((t, e, fl[0], fl[1], fl[2]))
        a = np.array(rows, dtype=np.float64)
        return a[:, 0].astype(np.int64), a[:, 1].astype(np.int64), a[:, 2:5].copy()


def field_at(P: np.ndarray, area: float, fluxes: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Evaluate sum_i F_i (r - P_i)/(2A) at points r [..., 3]."""
    out = np.zeros(np.shape(r))
    for i in range(3):
        out = out + fluxes[i] * (r - P[i]) / (2.0 * area)
    return out
