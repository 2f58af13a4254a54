"""CPU oracle for the sparse-tile lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing here is imported by the GPU
library or its Python binding, and nothing here imports them.

  dense      -- ctypes wrapper of ``lbm_oracle.c`` (plain FP64 dense LBM)
  tiles      -- NumPy tiling of a solid mask (Sec. 3 of the paper)
  perfmodel  -- the paper's overhead model (Eqs. 9-43)
  nn         -- layer operations of the warm-start network and their gradients
  invariants -- conserved quantities of the discrete step (mass per component,
                staggered momentum per axis component) and the projection of a
                starting state onto the values of a start from rest
"""
