"""MI355X (gfx950) state-vector sweep for random lattice circuits.

The compute path is libqsv.so (hand-written HIP kernels behind a C ABI,
include/qsv.h); `qsv` is its ctypes binding and `workloads` the seeded
synthetic inputs.
"""
from . import workloads  # noqa: F401
