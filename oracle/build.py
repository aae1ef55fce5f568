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
# No -march=native: the library built here also runs on other hosts.
CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
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


if __name__ == "__main__":
    build(force=True, verbose=True)
    sys.exit(0)
