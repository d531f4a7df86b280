"""Write plain_barrier_6649.npz: the FP64 oracle's full run of the
plain-method workload (square barrier r = 0.6, V0 = E0/2, 48^3 FFT grid with
an 8-cell absorber, k0 = pi/(4h) along +z, 6649 leapfrog steps of Eq.
PSTDupdating from rest, box planes at indices 10 and 38, phasors of Eqs.
psiphasor / dpsiphasor over the last 1354 steps, normalised as in Eq.
scaledphsiphasor at the origin).  The potential is first rounded to float32,
the precision the library receives it in, so that the stored run and the
float32 path start from the same numbers.  Calls only oracle/ and synth/
(seeded inputs), with the oracle's default library-free transform.

    python tests/golden/make_plain_barrier_reference.py

Stored: psi = psi^6649 and psi_prev = psi^6648 ([k][j][i] complex128), phi and
dphi (six faces x 48 x 48, in the face order x-lo, x-hi, y-lo, y-hi, z-lo,
z-hi), the unnormalised incident phasor and the number of window steps.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import synth  # noqa: E402
from oracle import pstd as opstd  # noqa: E402

OUT = os.path.join(HERE, "plain_barrier_6649.npz")


def main():
    prob, V = synth.plain_barrier()
    V = V.astype(np.float32).astype(np.float64)
    model = opstd.build(prob, V)
    shape = (prob.n[2], prob.n[1], prob.n[0])
    prev = np.zeros(shape, np.complex128)
    cur = np.zeros(shape, np.complex128)
    sd = opstd.SurfaceDFT(model)
    t0 = time.time()
    for n in range(prob.n_steps):
        if prob.dft_begin <= n < prob.dft_end:
            sd.accumulate(cur, n)
        prev, cur = cur, opstd.step(model, prev, cur, n)
        if n % 500 == 0:
            print(f"step {n} of {prob.n_steps}, {time.time() - t0:.0f} s", flush=True)
    phi, dphi = sd.normalized()
    np.savez_compressed(OUT, psi=cur, psi_prev=prev, phi=np.stack(phi), dphi=np.stack(dphi),
                        inc=np.array(sd.inc), window_steps=np.array(sd.count), steps=np.array(prob.n_steps),
                        dft=np.array([prob.dft_begin, prob.dft_end]))
    print(f"wrote {OUT} after {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
