"""Writes tests/golden/sphere_scan_mie.json: the Mie-series monostatic RCS
(dBsm) of the unit PEC sphere at the electrical sizes of the sphere
frequency scan (kr from 10 to 12,000, 40 log-spaced values) and of the
ray-spacing study (kr = 1000).  Calls only the oracle's Mie series.

    python -m tests.golden.make_sphere_scan_mie
"""
import json
import os

import numpy as np

from oracle import mie

KR_SCAN = np.geomspace(10.0, 12000.0, 40)
KR_SPACING = 1000.0


def main():
    db = lambda kr: float(10.0 * np.log10(mie.mie_pec_backscatter_norm(kr) * np.pi))
    out = {"_source": "Mie series of the PEC sphere (oracle/mie.py), radius 1 m, sigma in dBsm",
           "kr_scan": KR_SCAN.tolist(), "mie_scan_dbsm": [db(k) for k in KR_SCAN],
           "kr_spacing": KR_SPACING, "mie_spacing_dbsm": db(KR_SPACING)}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere_scan_mie.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
