"""MI355X-native high occupancy multigrid (HOMG, arXiv:1108.2045).

The solver runs in the HIP library libhomg.so (C ABI in include/homg.h);
this package only loads it and marshals arguments.  Importing the package
does not touch the GPU; creating a Solver does.
"""
from .homg import (DIFFUSION_5PT_2D, JACOBI, LAPLACE_5PT_2D, LAPLACE_7PT_3D, LEARNED,  # noqa: F401
                   SMOOTHER_WEIGHTS, BatchSolver, HomgError, Solver, Trainer, learn_adam, learn_forward,
                   jacobi_weights, learn_grad, lib, residual_noalloc, version)
