"""Closed-form physical-optics RCS of canonical targets (textbook PO results
used to pin the oracle; none of them is printed in the paper, which names the
flat-plate formula only through the problem statement of the build).

TEST INFRASTRUCTURE ONLY.
"""
import numpy as np

C0 = 299_792_458.0


def plate_normal(area, freq_hz):
    """Flat plate at normal incidence: sigma = 4 pi A^2 / lambda^2."""
    lam = C0 / freq_hz
    return 4.0 * np.pi * area ** 2 / lam ** 2


def plate_principal_plane(a, b, freq_hz, theta_rad):
    """a x b plate tilted by theta about the side of length a (incidence in
    the plane containing side b and the normal):
    sigma = 4 pi (a b / lambda)^2 cos^2(theta) sinc^2(k b sin theta)."""
    lam = C0 / freq_hz
    k = 2.0 * np.pi / lam
    x = k * b * np.sin(theta_rad)
    s = np.sinc(x / np.pi)
    return 4.0 * np.pi * (a * b / lam) ** 2 * np.cos(theta_rad) ** 2 * s ** 2


def trihedral_square_peak(a, freq_hz):
    """Square trihedral on its symmetry axis: sigma = 12 pi a^4 / lambda^2,
    i.e. an effective flat-plate area of sqrt(3) a^2."""
    lam = C0 / freq_hz
    return 12.0 * np.pi * a ** 4 / lam ** 2


def dihedral_peak(a, b, freq_hz):
    """90-degree dihedral with a x b faces at its bisector:
    sigma = 8 pi a^2 b^2 / lambda^2 (effective area sqrt(2) a b)."""
    lam = C0 / freq_hz
    return 8.0 * np.pi * a ** 2 * b ** 2 / lam ** 2


def dbsm(s):
    return 10.0 * np.log10(s)
