"""Build libvrc.so, the HIP library of the VRC estimator, for gfx950.

Every source is compiled by hipcc into one shared library next to this file:

* ``-ffp-contract=off``: the traversal's crossing times must be computed as
  written (product, then sum), never fused into FMA, so that voxel sequences
  are reproducible operation by operation;
* ``-munsafe-fp-atomics``: floating-point atomic adds become the hardware
  ``global_atomic_add_f64/f32`` instructions instead of compare-and-swap
  loops;
* ``-Xclang -target-feature -Xclang -packed-fp32-ops``: no packed FP32
  instructions are generated.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvrc.so")
SOURCES = ["vrc_api.cpp", "vrc_xs.cpp", "vrc_tune.cpp", "vrc_serve.cpp", "vrc_walker.cpp", "vrc_kernels.hip",
           "vrc_sorted.hip", "vrc_batched.hip", "vrc_rz.hip"]
HEADERS = ["vrc_internal.h", "vrc_math.h", "vrc_device.h", os.path.join("..", "..", "include", "vrc.h")]
ARCH = os.environ.get("VRC_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: install ROCm or set HIPCC")


def flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        "-ffp-contract=off", "-munsafe-fp-atomics",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-command-line-argument",
    ]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libvrc.so: " + " ".join(cmd))
    if verbose and r.stderr.strip():
        # hipcc's host pass does not know the packed-fp32 feature; keep other warnings visible
        lines = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link libvrc.so."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    deps = srcs + [os.path.normpath(os.path.join(CSRC, h)) for h in HEADERS]
    if not force and os.path.exists(LIB):
        if os.path.getmtime(LIB) >= max(os.path.getmtime(p) for p in deps):
            return LIB
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.basename(s) + ".o") for s in srcs]
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as pool:
        list(pool.map(lambda so: _run([hipcc(), *flags(), "-c", so[0], "-o", so[1]], verbose), zip(srcs, objs)))
    tmp = LIB + ".tmp"
    _run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force=True, verbose=True)
