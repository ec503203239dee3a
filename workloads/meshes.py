"""Seeded, synthetic closed surface meshes (input generators only).

Every generator returns ``(xyz, tri)``: ``xyz`` float64 [n_v, 3] vertex
coordinates in metres and ``tri`` int32 [n_c, 3] vertex indices, each
triangle counter-clockwise when seen from outside (outward normal by the
right-hand rule).  The surfaces are closed, connected and orientable, which is
what the formulation assumes of the scatterer (Sec. II-A).  Nothing in this
module computes any part of the integral-equation method; it only builds the
geometry that both the HIP path and the oracle receive as input.
"""
from __future__ import annotations

import numpy as np

_PHI = (1.0 + 5.0 ** 0.5) / 2.0


def _icosahedron():
    v = np.array(
        [
            [-1, _PHI, 0], [1, _PHI, 0], [-1, -_PHI, 0], [1, -_PHI, 0],
            [0, -1, _PHI], [0, 1, _PHI], [0, -1, -_PHI], [0, 1, -_PHI],
            [_PHI, 0, -1], [_PHI, 0, 1], [-_PHI, 0, -1], [-_PHI, 0, 1],
        ],
        dtype=np.float64,
    )
    f = np.array(
        [
            [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
            [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
            [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
            [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
        ],
        dtype=np.int64,
    )
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


def icosphere(subdivisions: int, radius: float = 1.0):
    """Icosahedron refined ``subdivisions`` times by edge midpoints, each new
    vertex projected onto the sphere.  Level s has 10*4^s+2 vertices,
    30*4^s edges and 20*4^s triangles (s=2: 162/480/320, s=4: 2562/7680/5120)."""
    v, f = _icosahedron()
    verts = [tuple(p) for p in v]
    for _ in range(int(subdivisions)):
        cache: dict[tuple[int, int], int] = {}

        def mid(a: int, b: int) -> int:
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                p = (np.asarray(verts[a]) + np.asarray(verts[b])) * 0.5
                p /= np.linalg.norm(p)
                verts.append(tuple(p))
                idx = len(verts) - 1
                cache[key] = idx
            return idx

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        f = np.asarray(nf, dtype=np.int64)
    xyz = np.asarray(verts, dtype=np.float64) * float(radius)
    return xyz, f.astype(np.int32)


def geodesic_sphere(freq: int, radius: float = 1.0):
    """Class-I geodesic sphere: every icosahedron face split into freq^2
    triangles on a barycentric grid, vertices projected onto the sphere.
    10*freq^2+2 vertices, 30*freq^2 edges, 20*freq^2 triangles."""
    n = int(freq)
    v0, f0 = _icosahedron()
    keymap: dict[tuple, int] = {}
    verts: list[np.ndarray] = []

    def vid(face_vertices, i, j):
        # lattice point i*(B-A)/n + j*(C-A)/n, keyed by the integer weights on
        # the icosahedron vertex ids so that shared edges/vertices coincide
        a, b, c = face_vertices
        wa, wb, wc = n - i - j, i, j
        items = sorted(((int(a), wa), (int(b), wb), (int(c), wc)))
        key = tuple((x, w) for x, w in items if w != 0)
        idx = keymap.get(key)
        if idx is None:
            p = (wa * v0[a] + wb * v0[b] + wc * v0[c]) / n
            p = p / np.linalg.norm(p)
            verts.append(p)
            idx = len(verts) - 1
            keymap[key] = idx
        return idx

    tris = []
    for fv in f0:
        for i in range(n):
            for j in range(n - i):
                p00 = vid(fv, i, j)
                p10 = vid(fv, i + 1, j)
                p01 = vid(fv, i, j + 1)
                tris.append([p00, p10, p01])
                if i + j < n - 1:
                    p11 = vid(fv, i + 1, j + 1)
                    tris.append([p10, p11, p01])
    xyz = np.asarray(verts, dtype=np.float64) * float(radius)
    return xyz, np.asarray(tris, dtype=np.int32)


def torus(major: float, minor: float, n_u: int, n_v: int):
    """Torus about the z axis on an n_u x n_v (toroidal x poloidal) grid, each
    quad split into two triangles: n_u*n_v vertices, 3*n_u*n_v edges and
    2*n_u*n_v triangles; genus 1, so two global loops."""
    u = 2.0 * np.pi * np.arange(n_u) / n_u
    w = 2.0 * np.pi * np.arange(n_v) / n_v
    uu, ww = np.meshgrid(u, w, indexing="ij")
    rr = major + minor * np.cos(ww)
    xyz = np.stack([rr * np.cos(uu), rr * np.sin(uu), minor * np.sin(ww)], axis=-1)
    xyz = xyz.reshape(-1, 3)

    def idx(i, j):
        return (i % n_u) * n_v + (j % n_v)

    tris = []
    for i in range(n_u):
        for j in range(n_v):
            a, b, c, d = idx(i, j), idx(i + 1, j), idx(i + 1, j + 1), idx(i, j + 1)
            tris.append([a, b, c])
            tris.append([a, c, d])
    return xyz.astype(np.float64), np.asarray(tris, dtype=np.int32)


def cube(edge: float, n: int):
    """Surface of an axis-aligned cube of side ``edge`` centred at the origin,
    each face an n x n grid of squares split into two triangles:
    6n^2+2 vertices, 18n^2 edges, 12n^2 triangles."""
    h = edge / 2.0
    keymap: dict[tuple, int] = {}
    verts: list[tuple] = []

    def vid(p):
        key = tuple(int(round((x + h) / edge * n)) for x in p)
        idx = keymap.get(key)
        if idx is None:
            verts.append(tuple(-h + edge * k / n for k in key))
            idx = len(verts) - 1
            keymap[key] = idx
        return idx

    tris = []
    for axis in range(3):
        for sgn in (-1.0, 1.0):
            a1, a2 = (axis + 1) % 3, (axis + 2) % 3
            for i in range(n):
                for j in range(n):
                    def pt(ii, jj):
                        p = [0.0, 0.0, 0.0]
                        p[axis] = sgn * h
                        p[a1] = -h + edge * ii / n
                        p[a2] = -h + edge * jj / n
                        return vid(p)
                    q00, q10, q11, q01 = pt(i, j), pt(i + 1, j), pt(i + 1, j + 1), pt(i, j + 1)
                    # (a1, a2, axis) is right-handed, so q00->q10->q11 is CCW
                    # seen from +axis; flip on the negative face
                    if sgn > 0:
                        tris += [[q00, q10, q11], [q00, q11, q01]]
                    else:
                        tris += [[q00, q11, q10], [q00, q01, q11]]
    return np.asarray(verts, dtype=np.float64), np.asarray(tris, dtype=np.int32)


def tetrahedron(scale: float = 1.0):
    """Regular tetrahedron: 4 vertices, 6 edges, 4 triangles."""
    xyz = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    xyz *= scale / np.sqrt(3.0)
    tri = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]], dtype=np.int32)
    return xyz, tri


def outward_volume(xyz: np.ndarray, tri: np.ndarray) -> float:
    """Signed enclosed volume (positive for outward orientation)."""
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)
