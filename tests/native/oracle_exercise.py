"""Exercises the oracle's entry points (run in a subprocess by
tests/test_sanitizers.py with the library built under AddressSanitizer and
UndefinedBehaviorSanitizer, selected by SSTEP_ORACLE_LIB)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import gen  # noqa: E402
import oracle  # noqa: E402

pr = gen.small_faces3d(7, 6, 5, seed=1)
A = oracle.problem_csr(pr)
b = oracle.spmv(A, pr.xstar)
out = oracle.solve(A, b, None, 6, 10, pr.lmin, pr.lmax, 1e-10, hist_cap=500)
assert out["status"] == 0, out["status"]
oracle.step(A, b, np.zeros(pr.n), 6, 10, pr.lmin, pr.lmax, want_basis=True)
oracle.step(A, b, np.zeros(pr.n), 4, 3, pr.lmin, pr.lmax, basis="monomial", precond=0, p0_mode=1)
oracle.lanczos(A, gen.uniform(gen.rng(2), pr.n), 12)
oracle.grad_faces(*pr.dims, out["x"], out["x"])
oracle.grad_csr(A, out["x"], out["x"])
oracle.assemble_stencil27(5, 4, 3)
tl = gen.two_level(3, nc=(3, 4, 2))
oracle.coarse_fgs(tl.nc, tl.kx, tl.ky, tl.kz, tl.f, 5)
# argument errors and edge cases
assert oracle.solve(A, b, None, 0, 10, pr.lmin, pr.lmax, 1e-8)["status"] == 1
assert oracle.solve(A, np.zeros(pr.n), None, 4, 5, pr.lmin, pr.lmax, 1e-8)["iters"] == 0
assert oracle.lanczos(A, np.zeros(pr.n), 5)["m"] == 0
bad = (A[0], A[1].copy(), A[2])
bad[1][3] = pr.n + 5
assert not oracle.csr_valid(pr.n, bad)
print("oracle exercised")
