"""MI355X-native sheared mesoscale blob simulation (arXiv 1808.06381).

The step runs in hand-written HIP kernels behind the C ABI declared in
include/sim.h (libsim.so); ``paper_1808_06381_amd.sim`` is the thin ctypes
binding with the same names.  Importing the package loads nothing native.
"""
__all__ = ["inputs", "sim"]
