"""Far field of the transient current vs the Mie series (oracle; tests only).

Validation of Sec. V: the current is Fourier transformed and its scattered
far field compared with the Mie series of a PEC sphere.  The Mie series is the
textbook closed form (Bohren & Huffman, "Absorption and Scattering of Light by
Small Particles", 1983, Sec. 4.4, with the perfectly conducting limit
a_n = psi_n'(x)/xi_n'(x), b_n = psi_n(x)/xi_n(x)); spherical Bessel functions
come from scipy.  Bistatic cross section sigma = 4 pi |S|^2 / k^2 with S_2 in
the E-plane and S_1 in the H-plane, Theta the angle from the propagation
direction.
"""
from __future__ import annotations

import numpy as np
from scipy.special import spherical_jn, spherical_yn

from . import quadrature as Q


def mie_pec_rcs(ka: float, theta: np.ndarray, radius: float = 1.0):
    """(sigma_E, sigma_H) of a PEC sphere of radius ``radius`` at size
    parameter x = ka, for scattering angles theta (radians)."""
    x = float(ka)
    k = x / radius
    nmax = int(x + 4.05 * x ** (1 / 3) + 8)
    n = np.arange(1, nmax + 1)
    jn, jnp = spherical_jn(n, x), spherical_jn(n, x, derivative=True)
    yn, ynp = spherical_yn(n, x), spherical_yn(n, x, derivative=True)
    psi = x * jn
    dpsi = jn + x * jnp
    xi = x * (jn + 1j * yn)
    dxi = (jn + 1j * yn) + x * (jnp + 1j * ynp)
    a = dpsi / dxi
    b = psi / xi
    mu = np.cos(theta)
    pi_prev = np.zeros_like(mu)
    pi_cur = np.ones_like(mu)
    S1 = np.zeros_like(mu, dtype=complex)
    S2 = np.zeros_like(mu, dtype=complex)
    for i, nn in enumerate(n):
        if nn == 1:
            pi_n = np.ones_like(mu)
        else:
            pi_n = ((2 * nn - 1) / (nn - 1)) * mu * pi_cur - (nn / (nn - 1)) * pi_prev
            pi_prev, pi_cur = pi_cur, pi_n
        if nn == 1:
            pi_prev, pi_cur = np.zeros_like(mu), pi_n
        tau_n = nn * mu * pi_n - (nn + 1) * pi_prev
        c = (2 * nn + 1) / (nn * (nn + 1))
        S1 += c * (a[i] * pi_n + b[i] * tau_n)
        S2 += c * (a[i] * tau_n + b[i] * pi_n)
    return 4 * np.pi * np.abs(S2) ** 2 / k ** 2, 4 * np.pi * np.abs(S1) ** 2 / k ** 2


def rcs_from_current(asm, j: np.ndarray, wave, freq: float, directions: np.ndarray):
    """Bistatic cross section from the marching current.

    j [n_steps, ne] are the h_i coefficients (time t_i = i dt).  J(f) and the
    incident spectrum E0(f) (the pulse at the origin) are discrete Fourier
    sums over the same samples; sigma = k^2/(4 pi) |r x N|^2 / |E0|^2 with
    N = sum_n J_n/E0 int f_n e^{j k r.r'} ds' (eta = 1)."""
    from .excitation import pulse_value
    t = asm.topo
    ns = j.shape[0]
    times = np.arange(1, ns + 1) * asm.dt
    ph = np.exp(-2j * np.pi * freq * times)
    Jf = ph @ j
    E0 = ph @ pulse_value(wave, times - wave.t0)
    k = 2 * np.pi * freq
    bary, w = Q.radon7()
    Pc = t.xyz[t.tri]
    pts = np.einsum("qi,cik->cqk", bary, Pc)
    out = []
    for rhat in directions:
        phase = np.exp(1j * k * (pts @ rhat))  # [nc, q]
        N = np.zeros(3, dtype=complex)
        for b in range(3):
            f = t.tri_sign[:, b, None, None] * (pts - Pc[:, b, None, :]) / (2 * t.area[:, None, None])
            contrib = np.einsum("cqk,cq,q->ck", f, phase, w) * t.area[:, None]
            N += (Jf[t.tri_edge[:, b]][:, None] * contrib).sum(0)
        N /= E0
        rxN = np.cross(rhat, N)
        out.append(k * k / (4 * np.pi) * np.real(np.vdot(rxN, rxN)))
    return np.array(out)
