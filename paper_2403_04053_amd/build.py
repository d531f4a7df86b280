"""Build libpstd.so (HIP for gfx950) in the package directory.

    python paper_2403_04053_amd/build.py

Objects and the compiler's temporaries go to a temporary directory outside
the source tree, which is removed afterwards; only libpstd.so is written
here (through a temporary name, renamed when complete).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpstd.so")
# longest compile first, so the parallel jobs finish together
SOURCES = ["pass_inst0.hip", "pass_inst1.hip", "pass_inst2.hip", "pass_inst3.hip", "pass_inst4.hip", "pass_inst5.hip",
           "project.hip", "api.hip", "batch.hip", "adjoint.hip", "sphere.hip", "fdtd.hip", "pulse.hip", "pass.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # never emit packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    if jobs is None:
        jobs = max(1, min(8, os.cpu_count() or 1))
    work = tempfile.mkdtemp(prefix="pstd_build_")
    try:
        env = dict(os.environ, TMPDIR=work)
        objs = []
        procs = []
        for src in SOURCES:
            obj = os.path.join(work, src.replace(".hip", ".o"))
            cmd = ["hipcc", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, env=env)))
            objs.append(obj)
            if len(procs) >= jobs:
                _wait(procs.pop(0))
        for p in procs:
            _wait(p)
        tmp = os.path.join(work, "libpstd.so")
        cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True, env=env)
        staged = LIB + ".tmp"
        shutil.copyfile(tmp, staged)
        os.chmod(staged, 0o755)
        os.replace(staged, LIB)
    finally:
        shutil.rmtree(work, ignore_errors=True)
    return LIB


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    if p.returncode != 0:
        sys.stderr.write(text)
        raise RuntimeError(f"hipcc failed on {src}")
    noisy = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if noisy:
        sys.stderr.write("\n".join(noisy) + "\n")


if __name__ == "__main__":
    print(build(verbose=True))
