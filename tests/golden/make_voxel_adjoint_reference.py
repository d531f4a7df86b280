"""Write voxel_adjoint_48.npz: the FP64 oracle's misfit and gradient of the
voxel-potential workload's recipe on a 48^3 grid over the full 6000 steps
(synth.voxel_potential_48; 32 x 32 detector points at z = 3.0, spacing h):
J(V) = 1/2 sum_o (|exp(i k.r_o) + Psi_o|^2 - I_o)^2 with I_o the oracle's
total-field intensity of the hidden potential, and dJ/dV by the oracle's
discrete adjoint of Eq. PSTDupdating, the surface DFT and the box projection.
Both potentials are first rounded to float32, as the library receives them.
Calls only oracle/ and synth/; the FFT step comes from the oracle's library
backend (pocketfft).  Holds every forward state in memory (about 11 GB).

    python tests/golden/make_voxel_adjoint_reference.py [--workers W]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import synth  # noqa: E402
from oracle import adjoint as oadj  # noqa: E402
from oracle import fft as offt  # noqa: E402

OUT = os.path.join(HERE, "voxel_adjoint_48.npz")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=4)
    args = ap.parse_args()
    prob, V0, Vh = synth.voxel_potential_48()
    V0 = V0.astype(np.float32).astype(np.float64)
    Vh = Vh.astype(np.float32).astype(np.float64)
    pts = synth.fresnel_plane(32, prob.h[0], 3.0)
    t0 = time.time()
    with offt.backend("pocketfft", workers=args.workers):
        target = oadj.intensity(prob, Vh, pts)
        print(f"target intensity after {time.time() - t0:.0f} s", flush=True)
        J, grad = oadj.gradient(prob, V0, pts, target)
    np.savez_compressed(OUT, J=np.array(J), grad=grad, target=target, points=pts, steps=np.array(prob.n_steps))
    print(f"wrote {OUT} (J = {J:.12e}) after {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
