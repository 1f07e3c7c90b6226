"""MI355X (gfx950) library for the low-rank isogeometric Tucker TPCG solver.

The numerical work lives in libtk.so (HIP kernels + host C++ setup, C ABI
in include/tk.h); `tk` is its ctypes binding and `problem` builds library
objects from the seeded `workloads` recipes.
"""
from . import tk  # noqa: F401
