"""Pins of the oracle's Mie series (the validation reference of Sec. V-A)
against limits fixed by physics, independent of the series itself."""
import numpy as np

from oracle.mie import mie_pec_rcs


def test_rayleigh_limit_of_a_pec_sphere():
    """ka << 1: the sphere scatters as an electric dipole 4 pi a^3 E plus a
    magnetic dipole -2 pi a^3 H, so sigma = 4 pi a^2 (ka)^4 |f|^2 with
    f = cos(theta) - 1/2 in the E-plane and 1 - cos(theta)/2 in the H-plane
    (backscatter 9 pi a^2 (ka)^4); corrections are O((ka)^2)."""
    th = np.linspace(0.0, np.pi, 19)
    for radius in (1.0, 0.5):
        ka = 0.01
        sE, sH = mie_pec_rcs(ka, th, radius)
        pref = 4 * np.pi * radius ** 2 * ka ** 4
        wantE = pref * (np.cos(th) - 0.5) ** 2
        wantH = pref * (1 - 0.5 * np.cos(th)) ** 2
        scale = pref * 9 / 4
        assert np.abs(sE - wantE).max() < 1e-3 * scale
        assert np.abs(sH - wantH).max() < 1e-3 * scale
        assert abs(sE[-1] / (9 * np.pi * radius ** 2 * ka ** 4) - 1) < 1e-3


def test_both_planes_agree_forward_and_backward():
    """At theta = 0 and pi the E- and H-plane amplitudes coincide (the
    scattering plane is undefined there), for every size."""
    for ka in (0.3, 1.05, 4.0, 12.0):
        sE, sH = mie_pec_rcs(ka, np.array([0.0, np.pi]))
        assert np.allclose(sE, sH, rtol=1e-10)


def test_geometric_optics_backscatter():
    """ka >> 1: the backscatter of a PEC sphere tends to its shadow area
    pi a^2 (with a creeping-wave ripple that decays as ka grows)."""
    for ka in (40.0, 80.0):
        sE, _ = mie_pec_rcs(ka, np.array([np.pi]))
        assert abs(sE[0] / np.pi - 1) < 0.05
