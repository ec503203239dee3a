"""Pins of the oracle's operators, lag matrices and temporal bases
(Sec. II-C, III-B, III-C, IV-A)."""
import numpy as np
import pytest

from oracle import operators as O
from oracle import quadrature as Q
from workloads import meshes


@pytest.fixture(scope="module")
def asm():
    xyz, tri = meshes.icosphere(1)
    a = O.Assembly(xyz, tri, 0.15)
    a.build()
    return a


def test_gram_exact_degree2(asm):
    G3 = asm.gram(Q.tri3())
    G7 = asm.gram(Q.radon7())
    assert np.abs(G3 - G7).max() < 1e-14 * np.abs(G7).max() * 10


def test_yukawa_symmetry_definiteness(asm):
    Zs, Zh = asm.Zs, asm.Zh
    assert np.abs(Zs - Zs.T).max() == 0.0
    assert np.abs(Zh - Zh.T).max() < 1e-14 * np.abs(Zh).max()
    # e^{-kR}/R is a positive-definite kernel: -Z^s SPD, -Z^h PSD
    assert np.linalg.eigvalsh(-Zs).min() > 0
    assert np.linalg.eigvalsh(-Zh).min() > -1e-12 * np.abs(Zh).max()
    # the BC divergence factors through Lambda: P^{Sigma H} Z^h = Z^h P^{Sigma H} = 0
    PSH = asm.proj.PPSH
    assert np.abs(PSH @ Zh).max() < 1e-12 * np.abs(Zh).max()
    assert np.abs(Zh @ PSH).max() < 1e-12 * np.abs(Zh).max()


def test_mfie_yukawa_minus_static_is_order_kappa2(asm):
    """(K_{-j kappa} - K_0) = O(kappa^2) (Sec. III-C): halving kappa divides
    the matrix difference by 4."""
    M0 = asm._mfie_only(0.0)
    d = [np.linalg.norm(asm._mfie_only(k) - M0) for k in (0.2, 0.1, 0.05)]
    assert 3.6 < d[0] / d[1] < 4.4 and 3.8 < d[1] / d[2] < 4.2


def test_static_mfie_property(asm):
    """P^{Sigma H}(G/2 - M0) G^-1 (G/2 + M0) P^{Lambda H} = 0 (eq. property):
    holds up to discretisation error, far below the unprojected product."""
    M0 = asm._mfie_only(0.0)
    G = asm.G
    prod = (0.5 * G - M0) @ np.linalg.inv(G) @ (0.5 * G + M0)
    proj = asm.proj.PPSH @ prod @ asm.proj.PLH
    r1 = np.linalg.norm(proj) / np.linalg.norm(prod)
    assert r1 < 1e-3
    # ... and the residual shrinks under refinement (level 1 -> level 2)
    xyz, tri = meshes.icosphere(2)
    a2 = O.Assembly(xyz, tri, 0.05, K=1)
    G2, M2 = a2.gram(), a2._mfie_only(0.0)
    prod2 = (0.5 * G2 - M2) @ np.linalg.inv(G2) @ (0.5 * G2 + M2)
    r2 = np.linalg.norm(a2.proj.PPSH @ prod2 @ a2.proj.PLH) / np.linalg.norm(prod2)
    assert r2 < 0.7 * r1


def test_lag_sums_and_projector_structure(asm):
    K = asm.K
    # sum_k A_k = 0: a constant-in-time current induces no vector-potential EMF
    SA = sum(asm.A)
    assert np.abs(SA).max() < 1e-12 * np.abs(asm.A[0]).max()
    # partition of unity of h_0: sum_k C_k = G/2 + sum_j N_j
    SC = sum(asm.C)
    assert np.abs(SC - 0.5 * asm.G - asm.N.sum(0)).max() < 1e-11 * np.abs(SC).max()
    # ... and sum_j N_j is the static MFIE matrix M0 (independent static route)
    M0 = asm._mfie_only(0.0)
    assert np.abs(asm.N.sum(0) - M0).max() < 1e-3 * np.abs(M0).max()
    # the scalar-potential lag blocks are pure stars: P^{Lambda H} B_k = 0
    for k in range(K + 1):
        assert np.abs(asm.proj.PLH @ asm.B[k]).max() < 1e-12 * (1 + np.abs(asm.B[k]).max())


def test_shell_sum_is_static_vector_potential(asm):
    """sum_j V_j (shells dt) equals V from one shell wider than the body."""
    a2 = O.Assembly(asm.topo.xyz, asm.topo.tri, 10.0)
    V2, _, _ = a2.shells()
    assert np.abs(asm.V.sum(0) - V2[0]).max() < 1e-6 * np.abs(V2[0]).max()


def test_band_limit_of_slabs():
    """T_k = 0 for k > K (causality band of the retarded kernels)."""
    xyz, tri = meshes.icosphere(0)
    a = O.Assembly(xyz, tri, 0.3)
    K = a.K
    b = O.Assembly(xyz, tri, 0.3, K=K + 3)
    T = b.build()
    assert np.abs(T[K]).max() > 1e-6
    assert np.abs(T[K + 1:]).max() == 0.0


def _h0(t, dt):
    return np.where((t >= -dt) & (t < 0), 1 + t / dt, np.where((t >= 0) & (t <= dt), 1 - t / dt, 0.0))


def _q0(t, dt):
    x = t / dt
    return np.where((t >= -dt) & (t < 0), 0.5 * (x + 1) ** 2,
                    np.where((t >= 0) & (t < dt), 0.5 - x * x + x,
                             np.where((t >= dt) & (t <= 2 * dt), 0.5 * (x - 2) ** 2, 0.0)))


def test_temporal_bases():
    dt = 0.7
    t = np.linspace(-2 * dt, 4 * dt, 6001)
    q = _q0(t, dt)
    dq = np.gradient(q, t)
    # C^1: no jump in the derivative; q_i' = (h_i - h_{i+1})/dt (Remark, Sec. IV-B)
    assert np.abs(dq - (_h0(t, dt) - _h0(t - dt, dt)) / dt).max() < 5e-3
    # partition of unity of the shifted families
    s_h = sum(_h0(t - i * dt, dt) for i in range(-6, 10))
    s_q = sum(_q0(t - i * dt, dt) for i in range(-6, 10))
    assert np.abs(s_h - 1).max() < 1e-12 and np.abs(s_q - 1).max() < 1e-12


@pytest.mark.parametrize("k", [0, 1, 2, 5])
def test_shell_combinations_match_bases(k):
    """The per-shell polynomial combinations reproduce int phi(R) b(k dt - R) dR
    for the paper's h_0, h_0' and q_0, with a smooth test density phi."""
    dt = 0.3
    R = np.linspace(1e-9, 12 * dt, 240001)
    dR = R[1] - R[0]
    phi = np.exp(-R) * (1 + R)
    nsh = 12
    mom = np.zeros((nsh, 3))
    for j in range(nsh):
        sel = (R > j * dt) & (R <= (j + 1) * dt)
        x = R[sel] / dt - j
        for p in range(3):
            mom[j, p] = np.sum(phi[sel] * x ** p) * dR

    def sh(j):
        return mom[j] if 0 <= j < nsh else np.zeros(3)

    tau = k * dt - R
    q_direct = np.sum(phi * _q0(tau, dt)) * dR
    q_comb = O.q0_combine(sh(k), sh(k - 1), sh(k - 2))
    assert abs(q_direct - q_comb) < 2e-4 * (abs(q_direct) + 1e-3)
    hp = np.where((tau >= -dt) & (tau < 0), 1 / dt, np.where((tau >= 0) & (tau < dt), -1 / dt, 0.0))
    a_direct = -np.sum(phi * hp) * dR
    a_comb = O.h0_prime_combine(sh(k)[0], sh(k - 1)[0], dt)
    assert abs(a_direct - a_comb) < 2e-3 * (abs(a_direct) + 1e-3)
    m_direct = np.sum(phi * (_h0(tau, dt) + R * hp)) * dR
    m_comb = O.mfie_combine(sh(k)[0], sh(k - 1)[0], k)
    assert abs(m_direct - m_comb) < 2e-3 * (abs(m_direct) + 1e-3)
