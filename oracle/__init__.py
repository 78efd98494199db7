"""FP64 CPU oracle for the high occupancy multigrid (arXiv:1108.2045).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the product
library never does, and the two share no code.

  homg      -- the HOMG method step by step (C kernels in homg_oracle.c)
  textbook  -- an independent textbook V-cycle multigrid and dense assembly
               of A, used to pin the HOMG oracle to the discrete solution
"""
