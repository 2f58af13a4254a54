"""CPU oracle for the sparse-tile lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing here is imported by the GPU
library or its Python binding, and nothing here imports them.

  dense      -- ctypes wrapper of ``lbm_oracle.c`` (plain FP64 dense LBM)
  tiles      -- NumPy tiling of a solid mask (Sec. 3 of the paper)
  perfmodel  -- the paper's overhead model (Eqs. 9-43)
"""
