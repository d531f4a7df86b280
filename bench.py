"""Benchmark of the PSTD hot path on one MI355X.

Workload: the square-barrier scattering problem on a 128^3 interior inside a
16-cell absorber (FFT grid 160^3, FP32 step), k0 = pi/(4h), barrier radius
2.4, V0 = E0/2, spherical equivalence surface of radius 5.0 (64 x 128
nodes).  One step = the three pencil passes of the leapfrog (spectral
kinetic term, potential, TF/SF source, absorber) and the FP64 running DFT on
the sphere's interpolation shell: the whole timed region is inside the DFT
window, so every step does the surface accumulation.

Prints one JSON line (metric: Gcell-updates/s of the FP32 PSTD step).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per cell of each pass kernel (its own inputs and outputs,
# each touched once): x reads psi^n, writes L (with the potential term; V is
# read only on the taper's core box, 0.1 B per cell of the 160^3 grid); y
# reads psi^n and L, writes L; z reads psi^n, L, psi^{n-1} and writes psi^{n+1}
PASS_BYTES = {"x": 16, "y": 24, "z": 32}
STEP_BYTES = 28  # whole step: read psi^{n-1}, psi^n, V; write psi^{n+1}

# HBM traffic per launch of the pass kernels on the square-barrier workload at
# 160^3 and 288^3 (sphere surface, so the passes carry no plane sums), from
# rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE runs of this script (KiB per
# dispatch, scaled by what the same counters read for a plain copy of 512 MiB:
# FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  Valid only for the kernel sources whose
# SHA-256 is TRAFFIC_SRC_SHA256; otherwise traffic is reported as null.  Key:
# (N, N1, N2, pencils per workgroup, stage-B split M1, axis).
TRAFFIC_SRC_SHA256 = "078e2b9d4f8c41e42c9823dd5d69562aecef325df1aa1ad62c78b466b763c044"
TRAFFIC_KIB = {  # (fetch, write) KiB per launch
    (160, 8, 20, 16, 0, 0): (33260, 32001), (160, 8, 20, 16, 0, 1): (64168, 32000), (160, 8, 20, 16, 0, 2): (96273, 32000),
    (160, 10, 16, 8, 0, 0): (33374, 32000), (160, 10, 16, 8, 0, 1): (64211, 32172), (160, 10, 16, 8, 0, 2): (96290, 32084),
    (160, 10, 16, 16, 0, 0): (34391, 32000), (160, 10, 16, 16, 0, 1): (64167, 32000), (160, 10, 16, 16, 0, 2): (96287, 32000),
    (160, 10, 16, 32, 0, 0): (34676, 32000), (160, 10, 16, 32, 0, 1): (64170, 32000), (160, 10, 16, 32, 0, 2): (96299, 32000),
    (160, 16, 10, 16, 0, 0): (33638, 32000), (160, 16, 10, 16, 0, 1): (64183, 32000), (160, 16, 10, 16, 0, 2): (96319, 32000),
    (160, 20, 8, 16, 0, 0): (32659, 32000), (160, 20, 8, 16, 0, 1): (64194, 32000), (160, 20, 8, 16, 0, 2): (96327, 32000),
    (288, 12, 24, 8, 0, 0): (190064, 186625), (288, 12, 24, 8, 0, 1): (373548, 192534), (288, 12, 24, 8, 0, 2): (753359, 188168),
    (288, 12, 24, 8, 4, 0): (190616, 186625), (288, 12, 24, 8, 4, 1): (374073, 194021), (288, 12, 24, 8, 4, 2): (751713, 188196),
    (288, 12, 24, 16, 0, 0): (188175, 186624), (288, 12, 24, 16, 0, 1): (373482, 186624), (288, 12, 24, 16, 0, 2): (560241, 186624),
    (288, 16, 18, 16, 0, 0): (187502, 186624), (288, 16, 18, 16, 0, 1): (373487, 186624), (288, 16, 18, 16, 0, 2): (560242, 186624),
    (288, 16, 18, 32, 0, 0): (188611, 186641), (288, 16, 18, 32, 0, 1): (373545, 186624), (288, 16, 18, 32, 0, 2): (560284, 186624),
    (288, 18, 16, 16, 0, 0): (187467, 186624), (288, 18, 16, 16, 0, 1): (373501, 186624), (288, 18, 16, 16, 0, 2): (560263, 186624),
    (288, 24, 12, 8, 0, 0): (187454, 186624), (288, 24, 12, 8, 0, 1): (373513, 190755), (288, 24, 12, 8, 0, 2): (638001, 186635),
    (288, 24, 12, 16, 0, 0): (187334, 186626), (288, 24, 12, 16, 0, 1): (373488, 186624), (288, 24, 12, 16, 0, 2): (560285, 186624),
}
KERNEL_SOURCES = ("paper_2403_04053_amd/csrc/pass_kernel.hpp", "paper_2403_04053_amd/csrc/pass_variants.hpp",
                  "paper_2403_04053_amd/csrc/dft.hpp", "paper_2403_04053_amd/csrc/internal.hpp")


# The shell DFT of the spherical surface (r = 5, 64 x 128 nodes) on the same
# workload, per launch of a pair of steps, valid for the sphere sources whose
# SHA-256 is SHELL_TRAFFIC_SRC_SHA256.
SHELL_TRAFFIC_SRC_SHA256 = "096c8ff0f16b3049b5c82c4e5df49a22cd4d03da7f60d8548781d006e4618a7f"
SHELL_TRAFFIC_KIB = (13072, 5252)
SHELL_SOURCES = ("paper_2403_04053_amd/csrc/sphere.hip",)

# The same for the FDTD kernel on the 160^3 grid (key: grid edge), valid for
# the sources whose SHA-256 is FDTD_TRAFFIC_SRC_SHA256.
FDTD_TRAFFIC_SRC_SHA256 = "d5187277b6240dcdf890cd190e5854694aa3d4825e1b2721c82b8d95b56c0c03"
FDTD_TRAFFIC_KIB = {160: (105996, 32000)}
FDTD_SOURCES = ("paper_2403_04053_amd/csrc/fdtd.hip", "paper_2403_04053_amd/csrc/dft.hpp",
                "paper_2403_04053_amd/csrc/internal.hpp")


def kernel_src_sha256(sources=KERNEL_SOURCES):
    import hashlib
    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    for f in sources:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(tile, axis):
    """(fetch + write) bytes per launch, or None when not measured for these sources."""
    if TRAFFIC_SRC_SHA256 is None or kernel_src_sha256() != TRAFFIC_SRC_SHA256:
        return None
    kib = TRAFFIC_KIB.get((*tile, axis))
    return None if kib is None else 1024 * (kib[0] + kib[1])


def measured_step_traffic(tiles, sphere):
    """HBM bytes of one step (the three passes in the chosen tiles, plus half
    a pair of shell-DFT steps with the sphere) from the measured counters, or
    None when any of them is not measured for these sources."""
    total = 0
    for axis in range(3):
        t = measured_traffic(tuple(tiles[axis]), axis)
        if t is None:
            return None
        total += t
    if sphere:
        if SHELL_TRAFFIC_SRC_SHA256 is None or kernel_src_sha256(SHELL_SOURCES) != SHELL_TRAFFIC_SRC_SHA256:
            return None
        total += 1024 * (SHELL_TRAFFIC_KIB[0] + SHELL_TRAFFIC_KIB[1]) / 2
    return int(total)


def measured_fdtd_traffic(n):
    if FDTD_TRAFFIC_SRC_SHA256 is None or kernel_src_sha256(FDTD_SOURCES) != FDTD_TRAFFIC_SRC_SHA256:
        return None
    kib = FDTD_TRAFFIC_KIB.get(n)
    return None if kib is None else 1024 * (kib[0] + kib[1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--n", type=int, default=160, help="FFT grid length per axis")
    ap.add_argument("--surface", choices=["sphere", "box"], default="sphere",
                    help="single: equivalence surface (sphere r = 5 with a shell DFT, or the box planes at "
                         "N/2 -+ 40 with the plane sums inside the passes)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true",
                    help="single: skip the whole-grid comparison with the FP64 oracle (and the CPU baseline)")
    ap.add_argument("--parity-steps", type=int, default=64,
                    help="single: steps of the whole-grid comparison with the FP64 oracle")
    ap.add_argument("--no-288", action="store_true", help="single: skip the 288^3 line beside the 160^3 one")
    ap.add_argument("--workload", choices=["single", "batch", "adjoint", "project", "subdomain", "x3", "fdtd", "pulse"],
                    default="single",
                    help="single: the 160^3 square-barrier solve; batch: 64 uneven instances in one batch; "
                         "adjoint: misfit gradient of the 160^3 voxel potential (6000 steps)")
    ap.add_argument("--fd-voxels", type=int, default=64, help="adjoint: finite-difference check voxels")
    ap.add_argument("--fd-delta", type=float, default=1e-2, help="adjoint: FD step in units of E0")
    ap.add_argument("--adj-steps", type=int, default=6000, help="adjoint: forward steps of the misfit run")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="first run a plain FP32 copy kernel over this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2403_04053_amd as P
    import synth

    if args.copy_mb:
        # reads and writes exactly copy_mb MiB: the scale for FETCH_SIZE / WRITE_SIZE
        a = torch.ones(args.copy_mb * 2 ** 18, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "adjoint":
        return bench_adjoint(args)
    if args.workload == "project":
        return bench_project(args)
    if args.workload == "subdomain":
        return bench_subdomain(args)
    if args.workload == "x3":
        return bench_x3(args)
    if args.workload == "fdtd":
        return bench_fdtd(args)
    if args.workload == "pulse":
        return bench_pulse(args)

    prob, V = synth.square_barrier_160(n_fft=args.n)
    # the whole timed region sits inside the surface-DFT window
    prob = prob.replace(dft_begin=0, dft_end=10 ** 12)
    if args.surface == "sphere":
        # spherical equivalence surface of radius 5 (on grids under 160 points
        # the largest radius whose shell stays out of the absorber: 4.3 at 128)
        radius = min(5.0, round((args.n // 2 - 16 - 5) * prob.h[0], 6))
        prob = prob.replace(surface_kind=1, sphere_radius=radius, sphere_nodes=(64, 128))
        surface = f"spherical equivalence surface r={radius} (64x128 nodes, shell DFT every step)"
    else:
        surface = "box equivalence surface at N/2-+40 (plane DFT sums inside the passes every step)"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    s = P.Solver(prob, stream=stream)
    s.set_potential(V)
    cells = prob.cells
    tiles = s.autotune(reps=20)

    s.run(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    s.run(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    step_traffic = measured_step_traffic(tiles, args.surface == "sphere") if args.n == 160 else None
    gcells = cells * args.steps / (ms / 1e3) / 1e9

    # per-pass kernel durations, HIP events on the solver's stream
    n_timed = min(args.steps, 100)
    pass_ms = s.run_timed(n_timed)
    avg = {k: pass_ms[i] / n_timed for i, k in enumerate("xyz")}
    dom = max(avg, key=avg.get)
    # the dominant kernel's duration per launch: back-to-back launches
    # bracketed by HIP events on the solver's stream (the in-step events
    # above also hold the dispatch gap between kernels)
    dom_us = s.pass_time("xyz".index(dom), reps=100)
    # algorithmic bytes: the step's 28 B per cell-update (read psi^{n-1},
    # psi^n, V; write psi^{n+1}) over the dominant kernel's launch; the
    # kernel's own inputs and outputs (PASS_BYTES) are reported beside it
    achieved = STEP_BYTES * cells / (dom_us / 1e6) / 1e9
    own = PASS_BYTES[dom] * cells / (dom_us / 1e6) / 1e9
    finite = bool(torch.isfinite(torch.view_as_real(s.psi(0))).all().item())

    out = {
        "metric": "PSTD Gcell-updates/s (FP32 step, FP64 surface DFT)",
        "value": round(gcells, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"square barrier r=2.4 V0=E0/2, {args.n}^3 FFT grid ({args.n - 32}^3 inside a 16-cell absorber), "
                        f"k0=pi/(4h), TF/SF + absorber, {surface}",
            "grid": [args.n] * 3,
            "cells": cells,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"pass_{dom}",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            # the counters were taken on the sphere workload, whose passes carry no plane sums
            "traffic": (measured_traffic(tuple(tiles["xyz".index(dom)]), "xyz".index(dom))
                        if args.surface == "sphere" else None),
            "bytes_per_cell": STEP_BYTES,
            "kernel_us": round(dom_us, 3),
            "own_bytes_per_cell": PASS_BYTES[dom],
            "own_achieved": round(own, 1),
            "own_frac": round(own / HBM_PEAK_GBS, 4),
            "pass_ms_in_steps": {k: round(v, 5) for k, v in avg.items()},
            "tiles": {k: list(tiles[i]) for i, k in enumerate("xyz")},
            "step_frac_28B": round(STEP_BYTES * cells / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "step_traffic": step_traffic,
            "step_frac_measured": (round(step_traffic / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
                                   if step_traffic else None),
        },
        "wall_s": round(wall, 4),
        "finite": finite,
    }

    if not args.no_parity:
        # validity of the timed configuration: a whole-grid comparison with the
        # FP64 oracle over a few steps of this solver (the oracle's time is
        # the CPU baseline)
        parity, base = oracle_parity(s, prob, V, n0=3000, k_steps=args.parity_steps,
                                     with_baseline=not args.no_cpu_baseline)
        out["parity"] = parity
        out["valid"] = parity["ok"] and finite
        if base is not None:
            out["cpu_baseline"] = base
    s.close()
    del s
    if args.n == 160 and not args.no_288:
        out["hbm_resident_288"] = step_288(args, stream)
    print(json.dumps(out), flush=True)


def host_cpu():
    """(CPU model, logical CPUs of the machine, CPUs this process may use,
    threads the oracle's library transform uses)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    threads = min(usable, int(omp)) if omp and omp.isdigit() and int(omp) > 0 else usable
    return model, os.cpu_count(), usable, threads


def oracle_parity(s, prob, V, n0, k_steps, with_baseline):
    """Run k_steps of the benchmarked solver from a seeded state at step n0
    (source at full amplitude) and the same steps of the FP64 oracle; the
    whole-grid relative L2 difference of psi must be <= 1e-4.  The oracle's
    steps, timed on all usable host cores (library FFT threaded over the
    pencils), are the CPU baseline; one more step on one thread is reported
    beside it."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import fft as offt
    from oracle import pstd as opstd
    import synth
    V32 = np.asarray(V, dtype=np.float32).astype(np.float64)   # what the solver holds
    prev = synth.random_state(prob.n, 31).astype(np.complex64)
    cur = synth.random_state(prob.n, 32).astype(np.complex64)
    s.set_state(prev, cur, n0)
    s.run(k_steps)
    got = s.psi(0).cpu().numpy()
    model, ncpu, usable, threads = host_cpu()
    m = opstd.build(prob, V32)
    a, b = prev.astype(np.complex128), cur.astype(np.complex128)
    with offt.backend("pocketfft", workers=threads):
        t0 = time.perf_counter()
        for k in range(k_steps):
            a, b = b, opstd.step(m, a, b, n0 + k)
        dt = time.perf_counter() - t0
    rel = float(np.linalg.norm(got - b) / np.linalg.norm(b))
    parity = {"psi_rel_l2": rel, "bar": 1e-4, "ok": bool(rel <= 1e-4), "steps": k_steps, "from_step": n0,
              "state": "seeded complex normal psi^{n0-1}, psi^n0 (seeds 31, 32), rounded to complex64",
              "oracle": "FP64 numpy, FFT step from SciPy pocketfft"}
    if not with_baseline:
        return parity, None
    with offt.backend("pocketfft", workers=1), threadpool_limits(1):
        t1 = time.perf_counter()
        opstd.step(m, prev.astype(np.complex128), cur.astype(np.complex128), n0)
        dt1 = time.perf_counter() - t1
    base = {
        "value": round(prob.cells * k_steps / dt / 1e9, 6),
        "unit": "Gcell-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{k_steps} leapfrog steps of the {prob.n[0]}^3 grid from step {n0} (FP64 numpy oracle, "
                  f"FFT step from pocketfft with {threads} threads; elementwise work on one thread), {dt:.2f} s; "
                  f"these steps are also the parity check",
        "single_thread_value": round(prob.cells / dt1 / 1e9, 6),
        "cpu_model": model,
        "nproc": ncpu,
        "usable_cpus": usable,
    }
    return parity, base


def step_288(args, stream):
    """The same workload on a 288^3 FFT grid (256^3 inside the absorber,
    669 MB working set: beyond the 256 MB Infinity Cache, so the passes move
    their bytes to and from HBM), timed like the main line."""
    import torch

    import paper_2403_04053_amd as P
    import synth
    prob, V = synth.square_barrier_160(n_fft=288)
    prob = prob.replace(dft_begin=0, dft_end=10 ** 12, surface_kind=1, sphere_radius=5.0, sphere_nodes=(64, 128))
    s = P.Solver(prob, stream=stream)
    s.set_potential(V)
    tiles = s.autotune(reps=10)
    steps = 100
    s.run(16)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.run(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    us = {k: s.pass_time(i, reps=50) for i, k in enumerate("xyz")}
    dom = max(us, key=us.get)
    out = {
        "grid": [288] * 3,
        "value": round(prob.cells / (ms / 1e3) / 1e9, 3),
        "unit": "Gcell-updates/s",
        "ms_per_step": round(ms, 5),
        "step_frac_28B": round(STEP_BYTES * prob.cells / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "pass_us": {k: round(v, 2) for k, v in us.items()},
        "dominant": f"pass_{dom}",
        "frac_28B": round(STEP_BYTES * prob.cells / (us[dom] / 1e6) / 1e9 / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(tuple(tiles["xyz".index(dom)]), "xyz".index(dom)),
        "own_frac": round(PASS_BYTES[dom] * prob.cells / (us[dom] / 1e6) / 1e9 / HBM_PEAK_GBS, 4),
        "tiles": {k: list(tiles[i]) for i, k in enumerate("xyz")},
    }
    s.close()
    return out


def bench_batch(args):
    """64 instances with per-axis grid lengths in 96..192, random directions
    and energies, Gaussian-bump potentials, advanced together (grouped
    launches replayed from a HIP graph)."""
    import numpy as np
    import torch

    import paper_2403_04053_amd as P
    import synth
    inst = synth.uneven_batch()
    stream = torch.cuda.current_stream()
    b = P.Batch([p for p, _ in inst], stream=stream)
    for i, (_, V) in enumerate(inst):
        b.set_potential(i, V.astype(np.float32))
    b.autotune(reps=3)
    cells = sum(p.cells for p, _ in inst)
    b.run(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.run(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    out = {
        "metric": "PSTD Gcell-updates/s (FP32 step, batched uneven grids)",
        "value": round(cells * args.steps / (ms / 1e3) / 1e9, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "64 instances, per-axis FFT lengths 96..192, isotropic directions, "
                               "k0 in [pi/(8h), pi/(3h)], Gaussian bumps", "cells": cells},
    }
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    """Voxel-potential misfit on the 160^3 grid (128^3 interior): smoothed
    N(0, 0.1 E0) prior, target intensity of a hidden potential on a 128x128
    detector plane at z = 39.2 (spacing h), 6000 steps with the DFT window
    over all of them, sqrt(N) checkpoints.  Reports the backward / forward
    wall-time ratio and a central finite-difference check on seed-chosen
    core voxels."""
    import numpy as np
    import torch

    import paper_2403_04053_amd as P
    import synth
    prob, V0, Vh = synth.voxel_potential_160()
    N = args.adj_steps
    prob = prob.replace(dft_end=N)
    n_ck = max(1, math.ceil(math.sqrt(N)))
    pts = synth.fresnel_plane(128, prob.h[0], 39.2)
    stream = torch.cuda.current_stream()
    s = P.Solver(prob, stream=stream)
    tiles = s.autotune(reps=5)
    dev = torch.device("cuda:0")
    # target: total-field intensity of the hidden potential
    s.set_potential(Vh.astype(np.float32))
    s.run(N)
    psi = s.project(pts)
    r = torch.as_tensor(pts, dtype=torch.float64, device=dev)
    kh = torch.tensor([math.sin(prob.theta) * math.cos(prob.phi), math.sin(prob.theta) * math.sin(prob.phi),
                       math.cos(prob.theta)], dtype=torch.float64, device=dev)
    target = (torch.exp(1j * prob.k0 * (r @ kh)) + psi).abs() ** 2
    V = V0.astype(np.float32)
    s.set_potential(V)
    # first pair allocates the checkpoints
    s.misfit(N, pts, target, n_ck)
    s.misfit_gradient()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = s.misfit(N, pts, target, n_ck)
    t1 = time.perf_counter()
    g = s.misfit_gradient()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fwd, bwd = t1 - t0, t2 - t1
    # plain forward steps for reference
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.run(N)
    e1.record(stream)
    torch.cuda.synchronize()
    plain = e0.elapsed_time(e1) / 1e3
    g = g.cpu().numpy().astype(np.float64)
    out = {
        "metric": "adjoint/forward time ratio (misfit gradient vs misfit, sqrt(N) checkpoints)",
        "value": round(bwd / fwd, 4),
        "unit": "x",
        "n_gpus": 1,
        "steps": N,
        "warmup": 1,
        "ms_per_step": round(1e3 * bwd / N, 5),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "voxel potential (smoothed N(0, 0.1 E0) prior) on a 128^3 interior, 160^3 FFT grid, "
                               f"{N} steps, DFT window all steps, Fresnel plane 128x128 at z=39.2, "
                               f"{n_ck} checkpoints", "cells": prob.cells},
        "forward_s": round(fwd, 4),
        "backward_s": round(bwd, 4),
        "plain_steps_s": round(plain, 4),
        "forward_gcells": round(prob.cells * N / fwd / 1e9, 3),
        "J": J,
        "tiles": [list(t) for t in tiles],
    }
    if args.fd_voxels > 0:
        E0 = prob.k0 ** 2 / 2
        delta = args.fd_delta * E0
        worst = 0.0
        rows = []
        gmax = 0.0
        fds = []
        vox = synth.fd_voxels(prob, args.fd_voxels, 555)
        for i, v in enumerate(vox):
            Vp = V.copy()
            Vp[v] += delta
            Vm = V.copy()
            Vm[v] -= delta
            s.set_potential(Vp)
            Jp = s.misfit(N, pts, target, 1)
            s.set_potential(Vm)
            Jm = s.misfit(N, pts, target, 1)
            fds.append((Jp - Jm) / (2 * delta))
            print(f"fd {i + 1}/{len(vox)} voxel {v}: adjoint {g[v]:.6e} fd {fds[-1]:.6e}", file=sys.stderr, flush=True)
        fds = np.array(fds)
        ga = np.array([g[v] for v in vox])
        gmax = np.abs(fds).max()
        err = np.abs(ga - fds) / np.maximum(np.abs(fds), 1e-3 * gmax)
        out["fd_check"] = {"voxels": len(vox), "delta_E0": args.fd_delta, "max_rel_err": float(err.max()),
                           "median_rel_err": float(np.median(err)),
                           "criterion": "|g_adj - g_fd| / max(|g_fd|, 1e-3 max|g_fd|)"}
    print(json.dumps(out), flush=True)


def bench_pulse(args):
    """Pulsed incidence on the 160^3 square-barrier grid: a Gaussian packet
    (centre k = k0, width 6 reduced lengths) along z, the spherical surface
    of radius 5.6 accumulating phasors at five wavenumbers k = 0.8 ... 1.2
    k0 every step.  Reports the pulsed step rate (passes, the packet's
    table and layer-source kernels, the five-wavenumber shell DFT) and a
    whole solve (tau = 160, then the far field at every wavenumber) against
    the monochromatic solve of the same grid, which gives one wavenumber per
    run (14440 steps)."""
    import numpy as np
    import torch

    import paper_2403_04053_amd as P
    import synth
    # the pulsed sphere's shell must lie where the taper is zero: the 4-cell taper
    base, V = synth.square_barrier_160(n_fft=args.n, transition=4 if args.surface == "sphere" else 12)
    if args.surface == "sphere":
        sph = dict(surface_kind=1, sphere_radius=5.6 * args.n / 160, sphere_nodes=(64, 128))
        surf_txt = "sphere r=5.6 (64x128 nodes)"
    else:
        sph = {}
        surf_txt = "box planes N/2-+40 (plane values staged in the passes)"
    dtau_p, _ = P.pstd_reduced_step(P.problem_from(base))
    solve_steps = int(round(160.0 / dtau_p))
    prob = base.replace(n_steps=solve_steps, dft_begin=0, dft_end=10 ** 12, **sph)
    delta = base.k0 * base.h[0]
    psi0 = synth.gaussian_pulse_1d(512, delta, 1.0, 6.0, -30.0)
    kb = [0.8, 0.9, 1.0, 1.1, 1.2]
    stream = torch.cuda.current_stream()
    th = np.deg2rad(np.arange(0, 181, 1.0))
    ph = np.deg2rad(np.arange(0, 360, 2.0))
    T, F = np.meshgrid(th, ph, indexing="ij")
    dirs = torch.as_tensor(np.stack([np.sin(T) * np.cos(F), np.sin(T) * np.sin(F), np.cos(T)], -1).reshape(-1, 3),
                           device="cuda:0")

    def solve(problem, pulse, steps, tune=None):
        s = P.Solver(problem, stream=stream)
        s.set_potential(V)
        if tune is not None:
            for axis in range(3):
                s.set_tile(axis, tune[axis][1], tune[axis][3], tune[axis][4])
        else:
            tune = s.autotune(reps=20)
        if pulse:
            s.set_pulse(psi0, delta, kb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.run(steps)
        fs = [s.far_field(dirs, ik=ik) for ik in range(len(kb) if pulse else 1)]
        torch.cuda.synchronize()
        return s, time.perf_counter() - t0, tune

    # the pulsed step rate, inside the packet's passage
    s, _, tune = solve(prob, True, args.warmup)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.run(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cells = prob.cells
    n_timed = min(args.steps, 100)
    pass_ms = s.run_timed(n_timed)
    avg = {k: pass_ms[i] / n_timed for i, k in enumerate("xyz")}
    us = s.pass_time(2, reps=100)
    achieved = PASS_BYTES["z"] * cells / (us / 1e6) / 1e9
    finite = bool(torch.isfinite(torch.view_as_real(s.psi(0))).all().item())
    s.close()
    # whole solves: the pulsed one (five wavenumbers) and the monochromatic one
    s, t_pulse, _ = solve(prob, True, solve_steps, tune)
    s.close()
    cw_prob = base.replace(dft_begin=base.n_steps - 1354, dft_end=base.n_steps, **sph)
    # (the box's monochromatic solve keeps its plane sums inside the passes)
    s, t_cw, _ = solve(cw_prob, False, base.n_steps, tune)
    s.close()
    out = {
        "metric": "PSTD Gcell-updates/s (FP32 step, pulsed incidence, FP64 surface DFT at 5 wavenumbers)",
        "value": round(cells * args.steps / (ms / 1e3) / 1e9, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"square barrier r=2.4 V0=E0/2, {args.n}^3 FFT grid, Gaussian packet along z "
                               f"(k0, width 6), {surf_txt}, phasors at k/k0 = 0.8, 0.9, 1.0, 1.1, 1.2",
                   "cells": cells},
        "roofline": {"bound": "hbm", "kernel": "pass_z", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(tuple(tune[2]), 2) if args.n == 160 else None,
                     "bytes_per_cell": PASS_BYTES["z"], "kernel_us": round(us, 3),
                     "pass_ms_in_steps": {k: round(v, 5) for k, v in avg.items()}},
        "solve": {"pulsed_s": round(t_pulse, 3), "pulsed_steps": solve_steps, "wavenumbers": len(kb),
                  "monochromatic_s": round(t_cw, 3), "monochromatic_steps": base.n_steps,
                  "wavenumbers_per_s_pulsed": round(len(kb) / t_pulse, 3),
                  "wavenumbers_per_s_monochromatic": round(1 / t_cw, 3)},
        "finite": finite,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_pulse(prob, V, psi0, delta)
    print(json.dumps(out), flush=True)


def bench_subdomain(args):
    """The 288^3 Gaussian-bump workload (256^3 inside a 16-cell absorber) run
    as overlapping local-Fourier subdomains: 6^3 blocks of 48^3 cores with
    8-cell halos (local arrays of 64^3), on one GPU.  Rate in global cells;
    the local cells the passes transform are (64/48)^3 = 2.37 times more."""
    import numpy as np
    import torch

    import paper_2403_04053_amd as P
    import synth
    prob, V = synth.bumps_288()
    stream = torch.cuda.current_stream()
    s = P.Solver(prob, stream=stream)
    s.set_potential(V.astype(np.float32))
    tiles = s.autotune(reps=10)
    s.run(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.run(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cells = prob.cells
    local = cells * (64 / 48) ** 3
    pass_ms = s.run_timed(min(args.steps, 50))
    out = {
        "metric": "PSTD Gcell-updates/s, overlapping subdomains (global cells)",
        "value": round(cells * args.steps / (ms / 1e3) / 1e9, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "32 Gaussian bumps, 288^3 FFT grid (256^3 inside a 16-cell absorber), 6^3 subdomains "
                               "(core 48, halo 8, taper 3, local 64^3)", "cells": cells},
        "local_gcell_per_s": round(local * args.steps / (ms / 1e3) / 1e9, 3),
        "pass_ms_in_steps": {k: round(pass_ms[i] / min(args.steps, 50), 5) for i, k in enumerate("xyz")},
        "tiles": [list(t) for t in tiles],
    }
    print(json.dumps(out), flush=True)


def bench_fdtd(args):
    """The eighth-order FDTD variant of the step (Section 2.2.1) on the 160^3
    square-barrier grid (same physics, TF/SF box, absorber), no surface DFT:
    one stencil kernel per step.  Its algorithmic bytes are the step's floor,
    28 B/cell (read psi^n, psi^{n-1}, V; write psi^{n+1})."""
    import torch

    import paper_2403_04053_amd as P
    import synth
    prob, V = synth.square_barrier_160(n_fft=args.n)
    prob = prob.replace(scheme=1, dft_begin=0, dft_end=0)
    stream = torch.cuda.current_stream()
    s = P.Solver(prob, stream=stream)
    s.set_potential(V)
    s.autotune(reps=3)
    s.run(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.run(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cells = prob.cells
    us = s.pass_time(0, reps=100)
    achieved = STEP_BYTES * cells / (us / 1e6) / 1e9
    finite = bool(torch.isfinite(torch.view_as_real(s.psi(0))).all().item())
    out = {
        "metric": "FDTD-8 Gcell-updates/s (FP32 step)",
        "value": round(cells * args.steps / (ms / 1e3) / 1e9, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"square barrier r=2.4 V0=E0/2, {args.n}^3 grid, eighth-order FDTD step, TF/SF walls "
                               "+ absorber, no surface DFT", "cells": cells},
        "roofline": {"bound": "hbm", "kernel": "fdtd", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_fdtd_traffic(args.n), "bytes_per_cell": STEP_BYTES,
                     "kernel_us": round(us, 3)},
        "finite": finite,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_fdtd(prob, V)
    print(json.dumps(out), flush=True)


def bench_x3(args):
    """The paper's Section-4 run at its scale on one grid: central square
    potentials of radius 4 pi with s = 1, 0.5, -0.5, -1 at 20 points per
    wavelength (288^3, dtau = pi/1000, incidence along y; 36000 steps, 60000
    for the deep well), each solve timed whole; the far field, Psi at r_bar =
    2e4 and at r_bar = 100 against the exact partial-wave solution
    (solid-angle weighted rel-L2 over the x-y and y-z planes)."""
    import numpy as np
    import torch

    import paper_2403_04053_amd as P
    import synth

    # the exact partial-wave solution, stored by tests/golden/make_square_potential_reference.py
    root = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(root, "tests", "golden", "square_potential_reference.json")) as fh:
        gold = json.load(fh)

    def exact(sv, key):
        re_, im_ = gold["potentials"][str(sv)][key]
        v = np.asarray(re_) + 1j * np.asarray(im_)
        return np.concatenate([v, v])   # x-y and y-z planes

    g = np.deg2rad(np.asarray(gold["angles_deg"]))
    dirs = np.concatenate([np.stack([np.sin(g), np.cos(g), 0 * g], -1), np.stack([0 * g, np.cos(g), np.sin(g)], -1)])
    gam = np.concatenate([g, g])
    w = np.sin(gam) + 1e-2

    def rel(a, b):
        return math.sqrt(np.sum(w * np.abs(a - b) ** 2) / np.sum(w * np.abs(b) ** 2))

    stream = torch.cuda.current_stream()
    total_cells, total_s, acc = 0, 0.0, {}
    for sv, steps in ((1.0, 36000), (0.5, 36000), (-0.5, 36000), (-1.0, 60000)):
        prob, V = synth.x3_square_potential(sv, n_steps=steps)
        k = prob.k0
        sol = P.Solver(prob, stream=stream)
        sol.set_potential(V)
        sol.autotune(reps=5)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sol.run(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        total_s += e0.elapsed_time(e1) / 1e3
        total_cells += prob.cells * steps
        err = {"far": rel(sol.far_field(dirs).cpu().numpy(), exact(sv, "far"))}
        for rb in (2e4, 100.0):
            err[f"r{int(rb)}"] = rel(sol.project(dirs * (rb / k)).cpu().numpy(), exact(sv, f"r{int(rb)}"))
        acc[f"s={sv}"] = {kk: round(vv, 5) for kk, vv in err.items()}
        sol.close()
        print(f"x3 s={sv}: {steps} steps, {acc[f's={sv}']}", file=sys.stderr, flush=True)
    out = {
        "metric": "PSTD Gcell-updates/s, the paper's square potentials at its scale (288^3, 20 points per wavelength)",
        "value": round(total_cells / total_s / 1e9, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": 168000,
        "warmup": 0,
        "ms_per_step": round(1e3 * total_s / 168000, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "central square potential r_bar <= 4 pi, s = 1, 0.5, -0.5, -1; 288^3 FFT grid, dxb = "
                               "pi/10, dtau = pi/1000, 40-cell absorber, 41 SF cells, 12-cell taper, box on the SF "
                               "mid planes, incidence along y", "cells": 288 ** 3},
        "rel_l2_vs_partial_waves": acc,
        "solve_s": round(total_s, 2),
    }
    print(json.dumps(out), flush=True)


def bench_project(args):
    """The projection of the 160^3 square-barrier workload's box phasors: far
    field on the 181 x 360 grid of directions (1 degree), Fresnel plane of
    256 x 256 points at z = 7.2 (spacing h).  The phasors come from a short
    run with the window over all of it (their values do not change the
    cost).  The far field is one complex FP64 GEMM per face on the matrix
    cores, [directions x N_b] x [N_b x 2 N_c]."""
    import numpy as np
    import torch

    import paper_2403_04053_amd as P
    import synth
    prob, V = synth.square_barrier_160()
    prob = prob.replace(dft_begin=0, dft_end=10 ** 12)
    stream = torch.cuda.current_stream()
    s = P.Solver(prob, stream=stream)
    s.set_potential(V)
    s.run(200)
    th = np.deg2rad(np.arange(0, 181, 1.0))
    ph = np.deg2rad(np.arange(0, 360, 1.0))
    T, F = np.meshgrid(th, ph, indexing="ij")
    dirs = torch.tensor(np.stack([np.sin(T) * np.cos(F), np.sin(T) * np.sin(F), np.cos(T)], -1).reshape(-1, 3),
                        dtype=torch.float64, device="cuda")
    pts = torch.tensor(synth.fresnel_plane(256, prob.h[0], 7.2), dtype=torch.float64, device="cuda")

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ff_ms = timed(lambda: s.far_field(dirs), max(1, args.steps // 100))
    fr_ms = timed(lambda: s.project(pts), 1)
    # the same from the spherical surface of radius 5 (64 x 128 nodes)
    sp = P.Solver(prob.replace(surface_kind=1, sphere_radius=5.0, sphere_nodes=(64, 128)), stream=stream)
    sp.set_potential(V)
    sp.run(200)
    sff_ms = timed(lambda: sp.far_field(dirs), max(1, args.steps // 100))
    sfr_ms = timed(lambda: sp.project(pts), 1)
    nd = dirs.shape[0]
    n = prob.n
    # per face normal to axis a (in-plane axes b, c): M = directions, N = 2 N_c, K = N_b
    planes = [((1 if a == 0 else 0), (1 if a == 2 else 2)) for a in range(3)]
    gemm_flop = sum(2 * 8.0 * nd * (2 * n[c]) * n[b] for b, c in planes)
    out = {
        "metric": "NTDF projection time from the box (far field 181x360 directions, Fresnel 256x256 points), 160^3",
        "value": round(ff_ms + fr_ms, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": 200,
        "warmup": 1,
        "ms_per_step": None,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "square barrier 160^3 box phasors -> far field 65160 directions and Fresnel 65536 points "
                               "at z=7.2", "directions": nd, "points": int(pts.shape[0])},
        "far_field_ms": round(ff_ms, 4),
        "fresnel_ms": round(fr_ms, 4),
        "sphere_far_field_ms": round(sff_ms, 4),
        "sphere_fresnel_ms": round(sfr_ms, 4),
        "far_field_gemm_tflops_whole_call": round(gemm_flop / (ff_ms / 1e3) / 1e12, 3),
        "fp64_mfma_peak_tflops": 78.6,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline_fdtd(prob, V):
    """The FDTD-variant oracle, as it stands, on one full step of the grid."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import fdtd as ofdtd
    import synth
    m = ofdtd.build(prob, V)
    prev = np.zeros((prob.n[2], prob.n[1], prob.n[0]), np.complex128)
    cur = synth.random_state(prob.n, 1)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        ofdtd.step(m, prev, cur, 100)
        dt = time.perf_counter() - t0
    return {
        "value": round(prob.cells / dt / 1e9, 6),
        "unit": "Gcell-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"1 FDTD-8 step of the {prob.n[0]}^3 grid (FP64 numpy, single-threaded; host has "
                  f"{os.cpu_count()} logical CPUs), {dt:.2f} s",
    }


def cpu_baseline_pulse(prob, V, psi0, delta):
    """The pulsed-incidence oracle, as it stands, on one full step of the grid
    (the 1D packet's step, its deployment to the layer and the 3D step)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import pulse as opulse
    import synth
    pm = opulse.PulseModel(prob, V, psi0, delta)
    prev = np.zeros((prob.n[2], prob.n[1], prob.n[0]), np.complex128)
    cur = synth.random_state(prob.n, 1)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        pm.step(prev, cur, 100)
        pm.pulse.step()
        dt = time.perf_counter() - t0
    return {
        "value": round(prob.cells / dt / 1e9, 6),
        "unit": "Gcell-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"1 pulsed leapfrog step of the {prob.n[0]}^3 grid (FP64 numpy, library-free FFT, "
                  f"single-threaded; host has {os.cpu_count()} logical CPUs), {dt:.2f} s",
    }


if __name__ == "__main__":
    main()
