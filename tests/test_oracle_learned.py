"""Pins of the learned warm-start oracle: loop/star coordinates against the
decomposition's defining properties, the network gradient against central
finite differences, and Adam against its closed-form first step."""
import numpy as np
import pytest

from oracle import learned as Lr
from oracle.topology import Topology
from workloads import meshes


@pytest.fixture(scope="module", params=["sphere", "torus"])
def ls(request):
    if request.param == "sphere":
        xyz, tri = meshes.icosphere(1)
    else:
        xyz, tri = meshes.torus(1.0, 0.4, 10, 5)
    return Lr.LoopStar(Topology(xyz, tri))


def test_feature_count_and_harmonic_space(ls):
    t = ls.topo
    assert ls.nf == t.ne + 2  # Euler: N_V - N_E + N_C = 2 - N_H
    assert ls.nh == t.n_harmonic
    if ls.nh:
        assert np.allclose(ls.H.T @ ls.H, np.eye(ls.nh), atol=1e-12)
        # harmonic fields are both divergence- and curl-free in the discrete sense
        assert np.abs(ls.S.T @ ls.H).max() < 1e-10 and np.abs(ls.L.T @ ls.H).max() < 1e-10


def test_reconstruction_is_exact(ls):
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((5, ls.topo.ne))
    F = ls.features(Y)
    assert np.abs(ls.reconstruct(F) - Y).max() < 1e-10 * np.abs(Y).max()


def test_components_are_orthogonal(ls):
    rng = np.random.default_rng(4)
    y = rng.standard_normal(ls.topo.ne)
    f = ls.features(y)[0]
    z = np.zeros_like(f)
    parts = []
    for a, b in ((0, ls.nv), (ls.nv, ls.nv + ls.nc), (ls.nv + ls.nc, ls.nf)):
        g = z.copy()
        g[a:b] = f[a:b]
        parts.append(ls.reconstruct(g)[0])
    for i in range(3):
        for j in range(i + 1, 3):
            assert abs(parts[i] @ parts[j]) < 1e-10 * (y @ y)


def test_pure_star_and_pure_loop(ls):
    """y = Sigma s0 gives s = s0 - mean(s0) and nothing else; likewise loops."""
    rng = np.random.default_rng(5)
    s0 = rng.standard_normal(ls.nc)
    f = ls.features(ls.S @ s0)[0]
    assert np.abs(f[ls.nv:ls.nv + ls.nc] - (s0 - s0.mean())).max() < 1e-10
    assert np.abs(f[:ls.nv]).max() < 1e-10
    assert ls.nh == 0 or np.abs(f[ls.nv + ls.nc:]).max() < 1e-10
    l0 = rng.standard_normal(ls.nv)
    f = ls.features(ls.L @ l0)[0]
    assert np.abs(f[:ls.nv] - (l0 - l0.mean())).max() < 1e-10
    assert np.abs(f[ls.nv:]).max() < 1e-10


def _tiny():
    rng = np.random.default_rng(7)
    p = Lr.init_params(12, 9, 5, rng, out_scale=1.0)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.standard_normal(p[k].shape) * 0.1
    X = rng.standard_normal((6, 12))
    T = rng.standard_normal((6, 5))
    return p, X, T


def test_gradient_matches_central_differences():
    p, X, T = _tiny()
    _, g = Lr.loss_grad(p, X, T)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 7)):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = Lr.loss_grad(p, X, T)
            flat[idx] = old - h
            lm, _ = Lr.loss_grad(p, X, T)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[idx]) < 1e-7 * max(1.0, abs(fd)), (k, idx)


def test_zero_output_layer_is_quadratic_extrapolation():
    rng = np.random.default_rng(8)
    p = Lr.init_params(4 * 7, 6, 7, rng)
    p["W3"][:] = 0.0
    F = rng.standard_normal((9, 7))
    assert np.allclose(Lr.guess(p, F, 6), 3 * F[5] - 3 * F[4] + F[3], atol=1e-13)


def test_window_of_a_cubic_sequence():
    """Features following a cubic in the step index have constant third
    differences, so the target is exactly the normalised third difference
    and the input blocks are the normalised backward differences."""
    rng = np.random.default_rng(9)
    c = rng.standard_normal((4, 5))
    F = np.array([c[0] + c[1] * k + c[2] * k ** 2 + c[3] * k ** 3 for k in range(8)])
    x, t, rho3 = Lr.window(F, 6)
    d3 = 6.0 * c[3]  # third difference of a cubic
    assert np.isclose(rho3, np.sqrt(np.mean(d3 ** 2)))
    assert np.allclose(t, d3 / rho3)
    assert np.allclose(x[15:], d3 / rho3)
    assert np.allclose(x[:5], F[5] / np.sqrt(np.mean(F[5] ** 2)))


def test_adam_first_step_closed_form():
    """After one step from m = v = 0 the bias-corrected update is
    lr * g / (|g| + eps)."""
    p, X, T = _tiny()
    _, g = Lr.loss_grad(p, X, T)
    p0 = {k: v.copy() for k, v in p.items()}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    Lr.adam_step(p, g, m, v, 1, lr=1e-3, eps=1e-8)
    for k in p:
        assert np.allclose(p0[k] - p[k], 1e-3 * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-12, atol=1e-18)


def test_adam_second_step_scalar():
    """Scalar worked by hand: g1 = 2, g2 = -1, lr = 0.1, b1 = 0.5, b2 = 0.75,
    eps = 0.  m2 = 0.5*(0.5*2) + 0.5*(-1) = 0; so the second step is zero."""
    p = {"w": np.array([1.0])}
    m = {"w": np.zeros(1)}
    v = {"w": np.zeros(1)}
    Lr.adam_step(p, {"w": np.array([2.0])}, m, v, 1, lr=0.1, b1=0.5, b2=0.75, eps=0.0)
    assert np.isclose(p["w"][0], 0.9)
    Lr.adam_step(p, {"w": np.array([-1.0])}, m, v, 2, lr=0.1, b1=0.5, b2=0.75, eps=0.0)
    assert np.isclose(p["w"][0], 0.9)
