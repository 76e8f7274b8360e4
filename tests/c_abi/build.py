"""Build the C-ABI demo (step_demo.c) against libsim.so with gcc: a caller
that uses include/sim.h alone.  Writes tests/c_abi/step_demo."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
LIBDIR = os.path.join(ROOT, "paper_1808_06381_amd", "_lib")


def build(out=None, verbose=False):
    out = out or os.path.join(HERE, "step_demo")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "step_demo.c"), "-o", out, "-L", LIBDIR, "-lsim", "-lm",
           "-Wl,-rpath,$ORIGIN/../../paper_1808_06381_amd/_lib", "-Wl,-rpath," + LIBDIR,
           "-Wl,-rpath-link,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
