"""CPU oracle for the random lattice circuit state-vector sweep.

TEST INFRASTRUCTURE ONLY: a plain complex128 simulator, an independent
circuit generator and the branch split/combine reference.  Only tests/, the
smoke check and the benchmark's CPU-baseline leg may import it; the GPU
library never does.
"""
