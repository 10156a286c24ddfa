"""Shared test helpers: problem construction for both sides from the seeded
generators, and comparisons."""
from __future__ import annotations

import numpy as np

import gen
import oracle


def rel(a, b) -> float:
    """The larger of the norm-wise relative difference ||a - b|| / ||b|| and the
    entry-wise one max_i |a_i - b_i| / max_i |b_i|, so that a bound on it holds
    for the vector as a whole and for every entry on the vector's scale."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    d = np.abs(a - b)
    norm = float(np.linalg.norm(d) / max(np.linalg.norm(b), 1e-300))
    ent = float(d.max() / max(np.abs(b).max(), 1e-300)) if b.size else 0.0
    return max(norm, ent)


def oracle_rhs(pr):
    """b = A x* formed by the oracle (the HIP side receives this b)."""
    A = oracle.problem_csr(pr)
    return A, oracle.spmv(A, pr.xstar)


def make_operator(lib, pr, form: str):
    """Library operator for a generated problem: ``stencil`` (matrix-free,
    3D only) or ``csr`` (the generator's CSR arrays)."""
    if form == "stencil":
        if getattr(pr, "stencil", 7) == 27:
            return lib.Operator.stencil27(*pr.dims)
        return lib.Operator.stencil(*pr.dims, pr.kx, pr.ky, pr.kz)
    rp, ci, v = pr.csr()
    return lib.Operator.csr(rp, ci, v)


def ragged_poisson(seed=0, s=16, nu=25):
    """Constant Poisson on a ragged grid (several blocks plus a partial one)."""
    return gen.small_poisson3d(37, 29, 11, seed=seed, s=s, nu=nu)
