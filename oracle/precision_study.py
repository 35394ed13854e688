"""Precision and depth study (Sec. 6 discusses the single-precision phase
error after many reflections).  TEST INFRASTRUCTURE: it runs the oracle
twice on the same rays, once with its float64 path, distance D and phase
(the arithmetic the method is specified in here) and once with them in
float32, on a rectangular duct closed at the far end (rays entering at an
angle bounce between its walls up to ~36 times), and prints the phase error
k |D32 - D64| by bounce count and the relative deviation of A.

    python -m oracle.precision_study
"""
import numpy as np

import sbr_inputs as si
from . import oracle as O


def study(length, width, theta=84.0, phi=190.0, freq=10e9, bmax=64):
    V, T = si.duct(length, width, width, 24)
    m = O.Mesh(V, T)
    k0 = 2 * np.pi * freq / O.C0
    r64 = O.rcs_angle(m, theta, phi, [freq], 10.0, bmax=bmax, mode=O.MODE_PAPER)
    r32 = O.rcs_angle(m, theta, phi, [freq], 10.0, bmax=bmax, mode=O.MODE_PAPER, fp32_path=True)
    nb = r64["nb"]
    assert np.array_equal(nb, r32["nb"])  # the geometry is float32 in both
    err = k0 * np.abs(r32["D"] - r64["D"])
    rows = []
    for lo, hi in ((1, 2), (3, 10), (11, 20), (21, 64)):
        s = (nb >= lo) & (nb <= hi)
        if s.any():
            rows.append((lo, hi, int(s.sum()), float(np.sqrt((err[s] ** 2).mean())), float(err[s].max())))
    A64, A32 = r64["A"][0, 0, 0], r32["A"][0, 0, 0]
    return dict(rays=len(nb), max_bounces=int(nb.max()), rows=rows, dev=float(abs(A32 - A64) / abs(A64)))


def main():
    for L, w in ((6.0, 0.1), (60.0, 1.0)):
        r = study(L, w)
        print("duct %.0f m x %.1f m, 10 GHz: %d rays, up to %d bounces, |A32 - A64| / |A64| = %.2e"
              % (L, w, r["rays"], r["max_bounces"], r["dev"]))
        for lo, hi, n, rms, mx in r["rows"]:
            print("  N %2d-%2d: %7d rays, phase error rms %.2e rad, max %.2e rad" % (lo, hi, n, rms, mx))


if __name__ == "__main__":
    main()
