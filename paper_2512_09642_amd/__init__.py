"""MI355X-native s-step CG with forward Gauss-Seidel Gram solves.

Implements the hot path of S. Thomas and P. D'Ambra, "Inexact Gauss-Seidel
Coarse Solvers for AMG and s-step CG" (arXiv:2512.09642): the s-step CG outer
iteration on a sparse SPD system with a Chebyshev basis, tall-skinny Gram
reductions, column scaling and nu forward Gauss-Seidel sweeps, as HIP kernels
for gfx950 behind the C ABI of ``include/sstep.h``.  This package is the
argument-marshalling layer over that ABI; torch provides device memory and
streams.
"""
from ._native import SStepError, STATUS_NAMES, KT_NAMES, LIB_PATH, load  # noqa: F401
from .solver import BatchedSolver, CoarseSolver, Operator, Solver, SolveStats, require_gpu  # noqa: F401
from .autograd import SStepSolve, sstep_solve  # noqa: F401

__all__ = ["Operator", "Solver", "BatchedSolver", "CoarseSolver", "SolveStats", "SStepSolve", "sstep_solve", "SStepError", "require_gpu", "load"]
