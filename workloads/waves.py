"""Seeded incident-wave parameter sets and the named workload configurations.

Input generators only: directions, polarisations and pulse parameters are
drawn here and handed, as plain numbers, to both the HIP path and the oracle.
Units are the normalised ones used throughout the project: lengths in metres,
time measured as c*t in metres (c = 1), impedance eta = 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import meshes

C0 = 299792458.0  # m/s, used only to turn Hz into 1/m


@dataclass
class Wave:
    """One incident plane wave.

    pulse = 0 (modulated Gaussian):  e = A p cos(2 pi f0 u) exp(-u^2/(2 sig^2)),
        u = t - t0 - k.r, sig = 1/(2 pi bw), f0/bw in 1/m (cycles per metre of c*t).
    pulse = 1 (the Gaussian of the numerical-results section):
        e = (4A/(w sqrt(pi))) p exp(-((4/w)(t - t0 - k.r))^2).
    h = k x e (eta = 1).
    """

    k_hat: tuple
    pol: tuple
    amplitude: float = 1.0
    t0: float = 0.0
    pulse: int = 0
    w: float = 0.0
    f0: float = 0.0
    bw: float = 0.0


def mod_gauss_t0(bw: float, diameter: float) -> float:
    """Arrival delay that keeps |e| <= exp(-18) on the surface at t <= 0."""
    sig = 1.0 / (2.0 * np.pi * bw)
    return 6.0 * sig + diameter / 2.0


def pol_p1(k_hat: np.ndarray) -> np.ndarray:
    """First polarisation for direction k: normalize(a x k), a = z unless
    |k.z| > 0.9, then a = x."""
    k = np.asarray(k_hat, dtype=np.float64)
    a = np.array([0.0, 0.0, 1.0]) if abs(k[2]) <= 0.9 else np.array([1.0, 0.0, 0.0])
    p = np.cross(a, k)
    return p / np.linalg.norm(p)


def seeded_directions(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def batched_waves(n_dirs: int, seed: int, f0: float, bw: float, diameter: float,
                  both_pols: bool = True) -> list[Wave]:
    dirs = seeded_directions(n_dirs, seed)
    t0 = mod_gauss_t0(bw, diameter)
    out = []
    for k in dirs:
        p1 = pol_p1(k)
        out.append(Wave(tuple(k), tuple(p1), 1.0, t0, 0, 0.0, f0, bw))
        if both_pols:
            p2 = np.cross(k, p1)
            out.append(Wave(tuple(k), tuple(p2), 1.0, t0, 0, 0.0, f0, bw))
    return out


@dataclass
class Config:
    name: str
    mesh: tuple  # (xyz, tri)
    dt: float  # c*dt in metres
    n_steps: int
    waves: list = field(default_factory=list)


def hz_to_per_m(f_hz: float) -> float:
    return f_hz / C0


def sphere_small() -> Config:
    """Sphere r = 1 m, icosphere level 2 (480 edges), one x-polarised wave
    along -z, modulated Gaussian 50 MHz centre / 50 MHz bandwidth,
    c*dt = 0.05 m, 400 steps."""
    xyz, tri = meshes.icosphere(2)
    f0 = bw = hz_to_per_m(50e6)
    w = Wave((0.0, 0.0, -1.0), (1.0, 0.0, 0.0), 1.0, mod_gauss_t0(bw, 2.0), 0, 0.0, f0, bw)
    return Config("sphere-ico2-480e", (xyz, tri), 0.05, 400, [w])


def sphere_large() -> Config:
    """Sphere r = 1 m, icosphere level 4 (7680 edges), 150 MHz pulse,
    c*dt = 0.02 m, 2000 steps, single right-hand side."""
    xyz, tri = meshes.icosphere(4)
    f0 = bw = hz_to_per_m(150e6)
    w = Wave((0.0, 0.0, -1.0), (1.0, 0.0, 0.0), 1.0, mod_gauss_t0(bw, 2.0), 0, 0.0, f0, bw)
    return Config("sphere-ico4-7680e", (xyz, tri), 0.02, 2000, [w])


def torus_batched(n_dirs: int = 64) -> Config:
    """Torus R = 1 m, r = 0.3 m on an 80 x 25 grid (6000 edges), 64 seeded
    directions x 2 polarisations, 100 MHz pulse, c*dt = 0.03 m, 2000 steps."""
    xyz, tri = meshes.torus(1.0, 0.3, 80, 25)
    f0 = bw = hz_to_per_m(100e6)
    waves = batched_waves(n_dirs, 0, f0, bw, 2.6)
    return Config("torus-80x25-6000e-b128", (xyz, tri), 0.03, 2000, waves)


def small_case(kind: str = "ico1"):
    """Tiny meshes for oracle pins and fast parity tests."""
    if kind == "tet":
        return meshes.tetrahedron(1.0)
    if kind == "ico0":
        return meshes.icosphere(0)
    if kind == "ico1":
        return meshes.icosphere(1)
    if kind == "torus":
        return meshes.torus(1.0, 0.4, 10, 5)
    if kind == "cube":
        return meshes.cube(1.5, 2)
    raise ValueError(kind)


def uneven_batch(n: int = 32, seed: int = 0, n_dirs: int = 8):
    """32 seeded scatterers of uneven size marched together: type uniform over
    {sphere r = 1 m, cube of edge 1.5 m, torus (1 m, 0.3 m)}, edge count
    log-uniform in [500, 12000] (realised by the nearest geodesic frequency,
    cube grid or torus grid), 8 directions each with the first polarisation
    rule, 50 MHz pulse, c*dt = 0.05 m, 1500 steps."""
    rng = np.random.default_rng(seed)
    kinds = rng.integers(0, 3, size=n)
    sizes = np.exp(rng.uniform(np.log(500.0), np.log(12000.0), size=n))
    f0 = bw = hz_to_per_m(50e6)
    out = []
    for i, (kind, ne) in enumerate(zip(kinds, sizes)):
        if kind == 0:
            nu = max(4, int(round(np.sqrt(ne / 30.0))))
            xyz, tri = meshes.geodesic_sphere(nu, 1.0)
            diam, name = 2.0, "sphere-g%d" % nu
        elif kind == 1:
            m = max(5, int(round(np.sqrt(ne / 18.0))))
            xyz, tri = meshes.cube(1.5, m)
            diam, name = 1.5 * np.sqrt(3.0), "cube-%d" % m
        else:
            nv = max(4, int(round(np.sqrt(ne / (3.0 * 3.3)))))
            nu = max(8, int(round(3.3 * nv)))
            xyz, tri = meshes.torus(1.0, 0.3, nu, nv)
            diam, name = 2.6, "torus-%dx%d" % (nu, nv)
        t0 = mod_gauss_t0(bw, diam)
        ws = []
        for k in seeded_directions(n_dirs, 100 + i):
            ws.append(Wave(tuple(k), tuple(pol_p1(k)), 1.0, t0, 0, 0.0, f0, bw))
        out.append(Config(name, (xyz, tri), 0.05, 1500, ws))
    return out
