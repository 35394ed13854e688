"""Monostatic RCS of a perfectly conducting sphere from the Mie series.

TEST INFRASTRUCTURE ONLY (the analytic reference of the sphere validation,
Sec. 5.1).  The paper plots this curve but does not print the formula; the
textbook series used here is

    sigma / (pi a^2) = (ka)^-2 | sum_{n>=1} (-1)^n (2n+1) / (H_n(ka) H_n'(ka)) |^2

with H_n(x) = x h_n^(2)(x) the Riccati-Hankel function of the second kind and
H_n' its derivative.  It equals the usual (-1)^n (2n+1)(a_n - b_n) form
because the Riccati-Bessel Wronskian makes the numerator of a_n - b_n a unit
imaginary number.  The series is cut at n_max = ka + 4 (ka)^(1/3) + 10.
"""
import numpy as np
from scipy.special import spherical_jn, spherical_yn


def mie_pec_backscatter_norm(ka):
    """sigma / (pi a^2) for a PEC sphere of electrical size ka (scalar)."""
    ka = float(ka)
    nmax = int(ka + 4.0 * ka ** (1.0 / 3.0) + 10)
    n = np.arange(1, nmax + 1)
    j = spherical_jn(n, ka)
    y = spherical_yn(n, ka)
    jd = spherical_jn(n, ka, derivative=True)
    yd = spherical_yn(n, ka, derivative=True)
    h = j - 1j * y                     # spherical Hankel, second kind
    hd = jd - 1j * yd
    H = ka * h                         # Riccati-Hankel
    Hd = h + ka * hd                   # d/dx [x h_n(x)]
    s = np.sum(((-1.0) ** n) * (2 * n + 1) / (H * Hd))
    return float(np.abs(s) ** 2 / ka ** 2)


def mie_pec_sigma(radius, freq_hz, c=299_792_458.0):
    """Monostatic sigma in m^2."""
    k = 2.0 * np.pi * freq_hz / c
    return mie_pec_backscatter_norm(k * radius) * np.pi * radius ** 2
