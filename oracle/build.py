"""Build the CPU oracle shared library (plain C, gcc, no contraction of a*b+c).

TEST INFRASTRUCTURE ONLY: the library built here is loaded by the tests, the
smoke check and the benchmark's CPU-baseline leg, never by the GPU library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "_vrc_oracle.so")
SRC = [os.path.join(HERE, "vrc_oracle.c")]
DEPS = SRC + [os.path.join(HERE, "trav.inc")]

# -ffp-contract=off: no fused multiply-add, so the FP32/FP64 traversal is the
# exact IEEE sequence of operations the traversal reading prescribes.
# No -march=native here: the library built here also runs on other hosts
# (build_native() makes a copy for the host it runs on, for timing).
CFLAGS = ["-std=c11", "-O3", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-pthread", "-D_POSIX_C_SOURCE=200809L", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(p) for p in DEPS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, *SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_native(out_dir: str, verbose: bool = False) -> str:
    """The same library built for the host that runs this (-march=native), into out_dir."""
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, "_vrc_oracle_native.so")
    cmd = ["gcc", *CFLAGS, "-march=native", "-o", path, *SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return path


if __name__ == "__main__":
    build(force=True, verbose=True)
    sys.exit(0)
