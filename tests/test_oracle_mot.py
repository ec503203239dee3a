"""Pins of the oracle's marching scheme (Sec. IV-B, V)."""
import numpy as np
import pytest

from oracle import excitation as E
from oracle import mot
from oracle import operators as O
from oracle.mie import mie_pec_rcs, rcs_from_current
from workloads import meshes, waves


def _wave(f0, diameter, k=(0.0, 0.0, -1.0), p=(1.0, 0.0, 0.0)):
    return waves.Wave(k, p, 1.0, waves.mod_gauss_t0(f0, diameter), 0, 0.0, f0, f0)


def test_march_is_block_forward_substitution():
    xyz, tri = meshes.icosphere(0)
    a = O.Assembly(xyz, tri, 0.2)
    T = a.build()
    r = E.rhs(a, _wave(0.1, a.D), 40)
    y = mot.march(T, r)
    yb = mot.block_solve(T, r)
    assert np.abs(y - yb).max() < 1e-11 * np.abs(yb).max()


def test_factored_history_equals_the_slabs():
    """The history sum formed from the raw lag matrices and the
    preconditioners (no T_k, difference quotient moved onto the history by
    summation by parts) equals sum_k T_k y_{i-k} with the assembled slabs: on
    random histories and on the history of an actual march (where the sum
    cancels across lags), with one and with three right-hand sides."""
    xyz, tri = meshes.icosphere(1)
    a = O.Assembly(xyz, tri, 0.1)
    T = a.build()
    K, n = T.shape[0] - 1, T.shape[1]
    p = a.proj
    rng = np.random.default_rng(11)
    cases = [[rng.standard_normal(n) for _ in range(K + 1)],
             [rng.standard_normal((n, 3)) for _ in range(K + 1)]]
    r = E.rhs(a, _wave(0.1, a.D), 60)
    y = mot.march(T, r)
    i = 50  # ring[k-1] = y_{i-k}, zero before the first step
    cases.append([y[i - k - 1] if i - k >= 1 else np.zeros(n) for k in range(1, K + 2)])
    for ring in cases:
        dense = sum(T[k] @ ring[k - 1] for k in range(1, K + 1))
        fact = mot.history_sum_factored(a.A, a.B, a.C, p.PLH, p.PS, a.dtn, a.PE, a.PM, ring)
        assert np.abs(fact - dense).max() <= 1e-11 * np.abs(dense).max()


def test_post_processing_from_q_basis():
    """eq. post_processing equals (P^{LH} + d~_t P^Sigma) y(t) at t_i, with y
    expanded in h_i P^{LH} + q_i P^Sigma and q_i' from the Sec. IV-A q_0."""
    rng = np.random.default_rng(3)
    n, N, dt, T0 = 5, 12, 0.3, 2.0
    PS = rng.standard_normal((n, n))
    PS = PS @ PS.T
    PLH = np.eye(n) - 0.1 * PS
    y = rng.standard_normal((N, n))

    def q0p(t):  # derivative of q_0 written from its definition
        x = t / dt
        return np.where((t >= -dt) & (t < 0), (x + 1) / dt,
                        np.where((t >= 0) & (t < dt), (1 - 2 * x) / dt,
                                 np.where((t >= dt) & (t <= 2 * dt), (x - 2) / dt, 0.0)))

    j = mot.currents(PLH, PS, dt / T0, y)
    for i in range(1, N + 1):
        ti = i * dt
        direct = PLH @ y[i - 1] + sum(T0 * q0p(ti - l * dt) * (PS @ y[l - 1]) for l in range(1, N + 1))
        assert np.abs(direct - j[i - 1]).max() < 1e-12 * (1 + np.abs(direct).max())


def test_late_time_decay_sphere():
    """qHP TD-CFIE on a sphere: after the pulse the current keeps decaying
    with no floor (Sec. V-A)."""
    xyz, tri = meshes.icosphere(1)
    a = O.Assembly(xyz, tri, 0.1)
    T = a.build()
    r = E.rhs(a, _wave(0.1, a.D), 1500)
    j = mot.currents(a.proj.PLH, a.proj.PS, a.dtn, mot.march(T, r))
    nj = np.linalg.norm(j, axis=1)
    peak = nj.max()
    assert nj[-1] < 1e-20 * peak
    blocks = nj[300:].reshape(-1, 100).max(1)
    assert np.all(np.diff(np.log10(blocks)) < 0.5)  # no sustained growth


def test_no_growth_torus():
    """Torus (two global loops): solution stays bounded and decays over
    thousands of steps (Sec. V-B)."""
    xyz, tri = meshes.torus(1.0, 0.4, 12, 6)
    a = O.Assembly(xyz, tri, 0.1)
    T = a.build()
    r = E.rhs(a, _wave(0.1, a.D), 3000)
    j = mot.currents(a.proj.PLH, a.proj.PS, a.dtn, mot.march(T, r))
    nj = np.linalg.norm(j, axis=1)
    assert nj[-500:].max() < 1e-12 * nj.max()
    blocks = nj[500:].reshape(-1, 250).max(1)
    assert np.all(blocks[1:] < 10 * blocks[:-1])


def test_companion_spectrum_inside_unit_circle():
    """Polynomial eigenvalues of the marching system lie strictly inside the
    unit circle (Sec. V-A, qHP TD-CFIE)."""
    xyz, tri = meshes.icosphere(0)
    a = O.Assembly(xyz, tri, 0.25)
    T = a.build()
    assert mot.companion_radius(T) < 1.0


def test_companion_radius_closed_forms():
    """Scalar recurrences: t0 y_i + t1 y_{i-1} = 0 decays by |t1/t0|; a
    two-lag recurrence whose characteristic polynomial
    lambda^2 - 2 r cos(theta) lambda + r^2 has the roots r e^{+-i theta};
    decoupled unknowns give the largest radius of the two."""
    T = np.array([[[2.0]], [[-1.5]]])
    assert abs(mot.companion_radius(T) - 0.75) < 1e-14
    # lambda^2 + (t1/t0) lambda + (t2/t0) = 0 with roots 0.6 e^{+-i 0.4}
    r, th = 0.6, 0.4
    T2 = np.array([[[1.0]], [[-2 * r * np.cos(th)]], [[r * r]]])
    assert abs(mot.companion_radius(T2) - r) < 1e-14
    # two decoupled unknowns: radius of the slower one
    Tb = np.zeros((2, 2, 2))
    Tb[0] = np.diag([1.0, 4.0])
    Tb[1] = np.diag([-0.3, -3.6])
    assert abs(mot.companion_radius(Tb) - 0.9) < 1e-14


def test_condition_1_closed_forms():
    """cond_1 of a diagonal matrix is max|d| / min|d|; of a 2x2 rotation,
    (|c| + |s|)^2.  cond_2 of a diagonal matrix is max|d| / min|d|, of a
    rotation 1, of the shear [[1, e], [0, 1]] the ratio of its singular values
    (sqrt(e^2 + 4) +- e) / 2."""
    assert abs(mot.condition_1(np.diag([2.0, -8.0, 0.5])) - 16.0) < 1e-12
    c, s_ = np.cos(0.3), np.sin(0.3)
    R = np.array([[c, -s_], [s_, c]])
    assert abs(mot.condition_1(R) - (abs(c) + abs(s_)) ** 2) < 1e-12
    assert abs(mot.condition_2(np.diag([2.0, -8.0, 0.5])) - 16.0) < 1e-12
    assert abs(mot.condition_2(R) - 1.0) < 1e-12
    e = 3.0
    hi, lo = (np.sqrt(e * e + 4) + e) / 2, (np.sqrt(e * e + 4) - e) / 2
    assert abs(mot.condition_2(np.array([[1.0, e], [0.0, 1.0]])) - hi / lo) < 1e-12


def test_far_field_against_mie_series():
    """Sphere, ka ~ 1: the transient current's far field at an in-band
    frequency matches the Mie series (Sec. V-A, Fig. farfield)."""
    xyz, tri = meshes.icosphere(2)
    dt = 0.05
    a = O.Assembly(xyz, tri, dt)
    T = a.build()
    f0 = waves.hz_to_per_m(50e6)
    w = _wave(f0, a.D)
    n_steps = 600
    r = E.rhs(a, w, n_steps)
    j = mot.currents(a.proj.PLH, a.proj.PS, a.dtn, mot.march(T, r))
    th = np.linspace(0.05, np.pi - 0.05, 13)
    kdir = np.array(w.k_hat)
    pdir = np.array(w.pol)
    hdir = np.cross(kdir, pdir)
    dE = np.array([np.cos(t) * kdir + np.sin(t) * pdir for t in th])
    dH = np.array([np.cos(t) * kdir + np.sin(t) * hdir for t in th])
    sE = rcs_from_current(a, j, w, f0, dE)
    sH = rcs_from_current(a, j, w, f0, dH)
    mE, mH = mie_pec_rcs(2 * np.pi * f0, th)
    errE = np.sqrt(np.mean((sE - mE) ** 2) / np.mean(mE ** 2))
    errH = np.sqrt(np.mean((sH - mH) ** 2) / np.mean(mH ** 2))
    assert errE < 0.05 and errH < 0.05, (errE, errH)


def _large_dt_parts(xyz, tri, dt):
    """Peak solenoidal and irrotational current of a march whose pulse the
    step resolves (f = 1 / (64 dt)), and cond_2(T_0)."""
    a = O.Assembly(xyz, tri, dt)
    T = a.build()
    f = 1.0 / (64.0 * dt)
    w = _wave(f, a.D)
    n = int(np.ceil((w.t0 + 12.0 / f) / dt)) + 50
    j = mot.currents(a.proj.PLH, a.proj.PS, a.dtn, mot.march(T, E.rhs(a, w, n)))
    return T.shape[0] - 1, np.abs(j @ a.proj.PLH.T).max(), np.abs(j @ a.proj.PS.T).max(), mot.condition_2(T[0])


def test_large_time_step_scaling_exponents():
    """Large time steps (c dt from 2 to 128 sphere diameters, K = 2, the pulse
    scaled with the step): a PEC's low-frequency current has a solenoidal part
    that tends to the magnetostatic limit, O(1), and an irrotational part
    (the charge) of O(ka), so their log-log slopes against dt are 0 and -1;
    the stabilised operator keeps cond_2(T_0) flat (Sec. IV-A, V-A: no
    large-time-step breakdown).  Dropping the 1/dt~ of the post-processing
    (eq. post_processing) or of the irrotational term of W^M moves a slope by
    a whole power."""
    xyz, tri = meshes.icosphere(1)
    dts = np.array([4.0, 16.0, 64.0, 256.0])
    parts = [_large_dt_parts(xyz, tri, dt) for dt in dts]
    assert all(p[0] == 2 for p in parts)
    loop, star, cond = (np.array([p[i] for p in parts]) for i in (1, 2, 3))
    s_loop = np.diff(np.log(loop)) / np.diff(np.log(dts))
    s_star = np.diff(np.log(star)) / np.diff(np.log(dts))
    assert np.all(np.abs(s_loop) < 0.01), s_loop
    assert np.all(np.abs(s_star + 1.0) < 0.03), s_star
    assert cond.max() / cond.min() < 1.1 and cond.max() < 5.0, cond
