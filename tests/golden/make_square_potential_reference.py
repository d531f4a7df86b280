"""Write square_potential_reference.json: the exact partial-wave solution
for the central square potentials of Section 4 (Eq. sphericalV: V = s E0 for
r_bar <= 4 pi; s = 1, 0.5, -0.5, -1), in the units of the 288^3 workload
(k0 = pi, radius 4), at polar angles 0, 2, ..., 180 degrees from the
incident direction: the far-field amplitude f and the scattered wave at
r_bar = 2e4 and r_bar = 100.  Calls only oracle/.

    python tests/golden/make_square_potential_reference.py
"""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from oracle import partial_waves as pw  # noqa: E402


def main():
    k = math.pi
    a = 4.0
    E0 = k * k / 2
    deg = np.arange(0, 181, 2.0)
    th = np.deg2rad(deg)
    out = {"source": "partial waves, oracle/partial_waves.py; Section 4, Eq. sphericalV",
           "k0": k, "radius": a, "angles_deg": deg.tolist(), "potentials": {}}
    for s in (1.0, 0.5, -0.5, -1.0):
        entry = {}
        f = pw.amplitude(k, a, s * E0, th)
        entry["far"] = [f.real.tolist(), f.imag.tolist()]
        for rb in (2e4, 100.0):
            v = pw.scattered_wave(k, a, s * E0, rb / k, th)
            entry[f"r{int(rb)}"] = [v.real.tolist(), v.imag.tolist()]
        out["potentials"][str(s)] = entry
    with open(os.path.join(HERE, "square_potential_reference.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
