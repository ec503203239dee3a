"""The int8 digit storage of the lag blocks (QHP_I8X4), modelled in numpy and
pinned by what its definition fixes: digits reconstruct the fixed-point value
exactly and stay in range, the stored value is within half a quantum, the
13 kept digit products reproduce the exact product of the stored values to
within the products left out, and a march with this storage on the torus
matches the FP64 march as closely as FP32 storage does."""
import numpy as np
import pytest
import scipy.linalg as sla

from tests import digits_model as dm


def test_digits_reconstruct_and_range():
    rng = np.random.default_rng(0)
    q = rng.integers(-int(dm.LIM), int(dm.LIM) + 1, size=200000)
    q[:6] = [0, 1, -1, int(dm.LIM), -int(dm.LIM), (1 << 20)]
    t = dm.split4(q)
    assert np.array_equal(((t[0] * 128 + t[1]) * 128 + t[2]) * 128 + t[3], q)
    assert np.abs(t[0]).max() <= 127
    assert max(np.abs(d).max() for d in t[1:]) <= 64


def test_fixed_point_half_quantum():
    rng = np.random.default_rng(1)
    v = rng.standard_normal((50, 300)) * np.logspace(-6, 3, 50)[:, None]
    v[3] = 0.0
    s = np.abs(v).max(axis=1) / 127.0
    q = dm.fixed(v, s[:, None])
    err = np.abs(v - dm.value(s[:, None], q))
    quantum = s[:, None] * 2.0 ** -21
    assert np.all(err <= 0.5 * quantum * (1 + 1e-9) + 1e-300)
    assert np.all(q[3] == 0)


def _exact(Qv, Yv):
    """sum_j Qv(i, j) Yv(j, n) in extended precision"""
    return (Qv.astype(np.longdouble) @ Yv.astype(np.longdouble)).astype(np.float64)


def test_product_within_dropped_terms():
    rng = np.random.default_rng(2)
    n, m, B = 40, 257, 5
    T = rng.standard_normal((1, n, m)) * rng.uniform(0.1, 10, (1, n, 1))
    Y = rng.standard_normal((m, B)) * rng.uniform(0.1, 10, (1, B))
    S, Q = dm.quantise_blocks(T)
    sy, qy = dm.quantise_columns(Y)
    got = dm.product(S[0], Q[0], sy, qy)
    ref = _exact(dm.value(S[0][:, None], Q[0]), dm.value(sy[None, :], qy))
    bound = dm.dropped_bound(S[0], sy, m) + 1e-15 * np.abs(ref).max()
    assert np.all(np.abs(got - ref) <= bound)
    # leaving out even the smallest kept product is seen far above that error
    t, u = dm.split4(Q[0]), dm.split4(qy)
    less = got - S[0][:, None] * sy[None, :] * 2.0 ** -28 * (t[1].astype(float) @ u[3].astype(float))
    assert np.abs(less - ref).max() > 30 * np.abs(got - ref).max()


@pytest.fixture(scope="module")
def torus():
    from oracle import excitation as E, mot, operators as O
    from workloads import meshes, waves
    xyz, tri = meshes.torus(1.0, 0.4, 12, 6)
    dt, n = 0.12, 150
    asm = O.Assembly(xyz, tri, dt)
    asm.build()
    ws = waves.batched_waves(2, 5, 0.1, 0.1, asm.D)[:3]
    r = np.stack([E.rhs(asm, w, n) for w in ws], axis=-1)
    y = mot.march(asm.T, r)
    return asm, r, y


def march_digits(T, r):
    """y_i = T_0^{-1}(r_i - sum_k T_k y_{i-k}) with digit-stored T_k (k >= 1)
    and digit-stored y_{i-k}, products as the matrix cores form them."""
    K = T.shape[0] - 1
    S, Q = dm.quantise_blocks(T[1:])
    lu = sla.lu_factor(T[0])
    y = np.zeros_like(r)
    reps = []
    for i in range(1, r.shape[0] + 1):
        b = r[i - 1].copy()
        for k in range(1, min(i - 1, K) + 1):
            sy, qy = reps[i - k - 1]
            b -= dm.product(S[k - 1], Q[k - 1], sy, qy)
        y[i - 1] = sla.lu_solve(lu, b)
        reps.append(dm.quantise_columns(y[i - 1]))
    return y


def test_digit_march_matches_fp64(torus):
    """Error of the digit-stored march on the torus (three waves, 150 steps)
    against the FP64 march, beside FP32 blocks with carried rounding and
    FP64 products."""
    from oracle import mot
    asm, r, y = torus
    j = mot.currents(asm.proj.PLH, asm.proj.PS, asm.dtn, y)
    jd = mot.currents(asm.proj.PLH, asm.proj.PS, asm.dtn, march_digits(asm.T, r))
    err = float(np.abs(jd - j).max() / np.abs(j).max())
    T32 = asm.T.copy()
    c = np.zeros_like(T32[0])
    for k in range(1, T32.shape[0]):
        v = asm.T[k] + c
        T32[k] = v.astype(np.float32).astype(np.float64)
        c = v - T32[k]
    j32 = mot.currents(asm.proj.PLH, asm.proj.PS, asm.dtn, mot.march(T32, r))
    err32 = float(np.abs(j32 - j).max() / np.abs(j).max())
    print("digit march err %.3e, FP32 carried %.3e" % (err, err32))
    assert err < 1e-6
    assert err < 10 * err32
