"""Write square_barrier_14440.npz: samples of the FP64 oracle's full run of
the 160^3 square-barrier workload (barrier r = 2.4, V0 = E0/2, 16-cell
absorber, k0 = pi/(4h) along +z, 14 440 leapfrog steps of Eq. PSTDupdating
from rest, phasors of Eqs. psiphasor / dpsiphasor over the last 1354 steps,
normalised as in Eq. scaledphsiphasor at the origin).  The whole run is too
large to store, so this keeps: psi^14440 on the planes through the centre
normal to y and to z, at 8192 seeded cells, and its squared norm; the
scattered-field phasors at the 64 x 128 nodes of the sphere of radius 5
(value and normal derivative, from the shell DFT and the Lagrange
interpolation of the oracle's sphere module); the box phasors (planes at
indices 40 and 120) at 1024 seeded points of each face.  The potential is
first rounded to float32, as the library receives it.  Calls only oracle/ and
synth/; the FFT step comes from the oracle's library backend (pocketfft).

    python tests/golden/make_square_barrier_reference.py [--workers W] [--checkpoint PATH]

--checkpoint keeps the state every 500 steps at PATH and resumes from it.
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import synth  # noqa: E402
from oracle import fft as offt  # noqa: E402
from oracle import pstd as opstd  # noqa: E402
from oracle import sphere as osph  # noqa: E402

OUT = os.path.join(HERE, "square_barrier_14440.npz")
N_SAMPLES = 8192
N_FACE = 1024


def sample_plan(prob):
    """Seeded sample cells of psi and points of each box face (i, j on the
    face's [row][col] layout)."""
    rng = np.random.default_rng(14440)
    n = prob.n
    cells = np.stack([rng.integers(0, n[2], N_SAMPLES), rng.integers(0, n[1], N_SAMPLES),
                      rng.integers(0, n[0], N_SAMPLES)], 1)             # (k, j, i)
    faces = []
    for f in range(6):
        a, _ = opstd.FACES[f]
        rows, cols = {0: (n[2], n[1]), 1: (n[2], n[0]), 2: (n[1], n[0])}[a]
        faces.append(np.stack([rng.integers(0, rows, N_FACE), rng.integers(0, cols, N_FACE)], 1))
    return cells, np.stack(faces)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--checkpoint", default=None)
    args = ap.parse_args()
    prob, V = synth.square_barrier_160()
    V = V.astype(np.float32).astype(np.float64)
    model = opstd.build(prob, V)
    sph = osph.Sphere(prob, 5.0, 64, 128)
    shape = (prob.n[2], prob.n[1], prob.n[0])
    prev = np.zeros(shape, np.complex128)
    cur = np.zeros(shape, np.complex128)
    sd = opstd.SurfaceDFT(model)
    shd = osph.ShellDFT(model, sph)
    start = 0
    if args.checkpoint and os.path.exists(args.checkpoint):
        ck = np.load(args.checkpoint)
        start = int(ck["n"])
        prev, cur = ck["prev"], ck["cur"]
        sd.phi = list(ck["phi"])
        sd.dphi = list(ck["dphi"])
        sd.inc = complex(ck["inc"])
        sd.count = int(ck["count"])
        shd.phi = ck["shell"]
        shd.inc = float(ck["shell_inc"])
        print(f"resumed at step {start}", flush=True)
    t0 = time.time()
    with offt.backend("pocketfft", workers=args.workers):
        for n in range(start, prob.n_steps):
            if prob.dft_begin <= n < prob.dft_end:
                sd.accumulate(cur, n)
                shd.accumulate(cur, n)
            prev, cur = cur, opstd.step(model, prev, cur, n)
            if (n + 1) % 500 == 0:
                print(f"step {n + 1} of {prob.n_steps}, {time.time() - t0:.0f} s", flush=True)
                if args.checkpoint:
                    tmp = args.checkpoint + ".tmp.npz"
                    np.savez(tmp, n=n + 1, prev=prev, cur=cur, phi=np.stack(sd.phi), dphi=np.stack(sd.dphi),
                             inc=np.array(sd.inc), count=np.array(sd.count), shell=shd.phi,
                             shell_inc=np.array(shd.inc))
                    os.replace(tmp, args.checkpoint)
    cells, face_pts = sample_plan(prob)
    phi, dphi = sd.normalized()
    fphi = np.stack([phi[f][face_pts[f, :, 0], face_pts[f, :, 1]] for f in range(6)])
    fdphi = np.stack([dphi[f][face_pts[f, :, 0], face_pts[f, :, 1]] for f in range(6)])
    node_v, node_d = sph.node_values(shd.normalized())
    c = prob.n[0] // 2
    np.savez_compressed(
        OUT, steps=np.array(prob.n_steps), dft=np.array([prob.dft_begin, prob.dft_end]),
        cells=cells, psi_cells=cur[cells[:, 0], cells[:, 1], cells[:, 2]],
        psi_plane_z=cur[c], psi_plane_y=cur[:, c, :], psi_norm2=np.array(np.vdot(cur, cur).real),
        node_psi=node_v, node_dpsi=node_d, face_points=face_pts, face_phi=fphi, face_dphi=fdphi,
        inc=np.array(sd.inc), shell_inc=np.array(shd.inc))
    print(f"wrote {OUT} after {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
