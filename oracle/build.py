"""Build the CPU oracle shared library (oracle/liboracle.so) with gcc.

Plain FP64 C, no FMA contraction and no fast-math, so the pair decision
r^2 < rc^2 is the IEEE result of the operations as written.  OpenMP spreads
the brute-force pair loop of the velocity correlation over threads (fixed
chunks, per-thread compensated sums added in thread order) and the row loops
of the solve's products and vector updates (one thread per output, sums
sequential): results do not depend on the thread count.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["oracle.c", "mpnn.c", "vv.c", "block.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-fopenmp", "-Wall", "-Wextra", "-o", LIB + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
