"""Seeded synthetic problem generators shared by the oracle and the HIP path.

This package defines problems only: grids, sparse operators assembled from their
finite-difference definition, coefficient fields, random vectors and the
closed-form spectral bounds of the Jacobi-preconditioned Poisson operator.  It
holds none of the s-step CG arithmetic (no SpMV, basis, Gram, Gauss-Seidel or
update), so that the oracle and the GPU path stay independent of each other.
"""
from .problems import *  # noqa: F401,F403
