"""Lanczos spectrum bounds on the GPU (through the C ABI) against the oracle.

The device runs the M-inner-product Lanczos recurrence (one SpMV and two
fixed-order reductions per step) and finds the Ritz values by bisection on
Sturm counts; the oracle runs the same recurrence with compensated sums and
takes the Ritz values from LAPACK's tridiagonal eigensolver.  alpha, beta and
the Ritz values agree to 1e-10 relative, entry by entry; the bounds with the
10% margin drive solves that reach 1e-8 like the oracle's with the same
bounds.
"""
import numpy as np
import pytest
import torch

import gen
import oracle
from helpers import make_operator, oracle_rhs, ragged_poisson, rel

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def t64(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def host(t):
    return t.detach().cpu().numpy()


CASES = {
    "poisson_ragged_stencil": (lambda: ragged_poisson(0), "stencil", 16, 25),
    "faces_stencil": (lambda: gen.small_faces3d(23, 17, 13, seed=2, sigma=1.0), "stencil", 8, 25),
    "faces_csr": (lambda: gen.small_faces3d(19, 21, 7, seed=3, sigma=0.5), "csr", 5, 20),
    "c1_csr_2d": (lambda: gen.config1(0), "csr", 8, 20),
    "poisson_s2_fp32": (lambda: gen.small_poisson3d(20, 18, 16, seed=4), "stencil", 2, 10),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("steps", [1, 10, 24])
def test_lanczos_matches_oracle(hip, name, steps):
    make, form, s, nu = CASES[name]
    pr = make()
    A = oracle.problem_csr(pr)
    u = gen.uniform(gen.rng(17), pr.n)
    ref = oracle.lanczos(A, u, steps)
    prec = "fp32ir" if name.endswith("fp32") else "fp64"
    with hip.Solver(make_operator(hip, pr, form), s, nu, pr.lmin, pr.lmax, precision=prec) as sv:
        got = sv.lanczos(t64(u), steps)
    assert got["m"] == ref["m"]
    for key in ("alpha", "beta", "ritz"):
        assert rel(got[key], ref[key]) <= 1e-10, (key, got[key], ref[key])


def test_lanczos_eigenvector_start_and_zero_start(hip):
    nx, ny, nz = 12, 10, 9
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    k = np.arange(nz)[:, None, None]
    v = (np.sin(np.pi * (i + 1) / (nx + 1)) * np.sin(np.pi * (j + 1) / (ny + 1))
         * np.sin(3 * np.pi * (k + 1) / (nz + 1))).ravel()
    lam = (6 - 2 * np.cos(np.pi / (nx + 1)) - 2 * np.cos(np.pi / (ny + 1)) - 2 * np.cos(3 * np.pi / (nz + 1))) / 6
    lo, hi = gen.jacobi_poisson_bounds(nx, ny, nz)
    with hip.Solver(hip.Operator.stencil(nx, ny, nz), 8, 20, lo, hi) as sv:
        got = sv.lanczos(t64(v), 10)
        assert got["m"] == 1 and abs(got["ritz"][0] - lam) <= 1e-13
        with pytest.raises(hip.SStepError) as e:
            sv.lanczos(t64(np.zeros(nx * ny * nz)), 10)
        assert e.value.name == "SSTEP_E_ARG"


@pytest.mark.parametrize("name", ["poisson_ragged_stencil", "faces_stencil", "c1_csr_2d"])
def test_lanczos_bounds_drive_the_solve(hip, name):
    """10 steps, 10% margin (Sec. 8 setup): the bounds equal the oracle's from
    its own Ritz values, and the solve with them reaches 1e-8 within 5% of the
    oracle's iteration count with the same bounds."""
    make, form, s, nu = CASES[name]
    pr = make()
    A, b = oracle_rhs(pr)
    u = gen.uniform(gen.rng(23), pr.n)
    ref = oracle.lanczos(A, u, 10)
    lo, hi = oracle.lanczos_bounds(ref["ritz"], 0.1)
    with hip.Solver(make_operator(hip, pr, form), s, nu, pr.lmin, pr.lmax) as sv:
        glo, ghi = sv.lanczos_bounds(t64(u), 10, 0.1)
        assert abs(glo - lo) <= 1e-10 * lo and abs(ghi - hi) <= 1e-10 * hi, (glo, lo, ghi, hi)
        x, st = sv.solve(t64(b), None, 1e-8)
    ro = oracle.solve(A, b, None, s, nu, glo, ghi, 1e-8)
    assert ro["status"] == 0 and st.status == 0
    assert abs(st.outer_iters - ro["iters"]) <= max(1, int(0.05 * ro["iters"])), (st.outer_iters, ro["iters"])
    assert np.linalg.norm(b - oracle.spmv(A, host(x))) / np.linalg.norm(b) <= 1e-8


def test_set_bounds_equals_fresh_setup(hip):
    """Replacing the bounds re-captures the outer-iteration graph: the solve is
    bitwise the one of a context set up with those bounds."""
    pr = gen.small_faces3d(15, 14, 13, seed=6)
    A, b = oracle_rhs(pr)
    op = make_operator(hip, pr, "stencil")
    with hip.Solver(op, 8, 25, 0.0, 2.0) as sv:
        sv.set_bounds(0.02, 1.9)
        x1, s1 = sv.solve(t64(b))
    with hip.Solver(make_operator(hip, pr, "stencil"), 8, 25, 0.02, 1.9) as sv:
        x2, s2 = sv.solve(t64(b))
    assert s1.outer_iters == s2.outer_iters and torch.equal(x1, x2)
    with hip.Solver(make_operator(hip, pr, "stencil"), 8, 25, 0.0, 2.0) as sv:
        for lo, hi in ((0.5, 0.5), (-0.1, 1.0), (0.0, float("nan"))):
            with pytest.raises(hip.SStepError):
                sv.set_bounds(lo, hi)


def test_lanczos_full_size_224(hip):
    """Ten steps on the 224^3 Poisson operator (11.2M unknowns) against the
    oracle: alpha, beta, Ritz values within 1e-10; every Ritz value inside the
    closed-form spectrum of M^{-1}A."""
    N = 224
    A = oracle.assemble_stencil7(N, N, N)
    u = gen.uniform(gen.rng(29), N ** 3)
    ref = oracle.lanczos(A, u, 10)
    lo, hi = gen.jacobi_poisson_bounds(N, N, N)
    with hip.Solver(hip.Operator.stencil(N, N, N), 16, 25, lo, hi) as sv:
        got = sv.lanczos(t64(u), 10)
    assert got["m"] == ref["m"] == 10
    for key in ("alpha", "beta", "ritz"):
        assert rel(got[key], ref[key]) <= 1e-10, (key, got[key], ref[key])
    assert got["ritz"][0] >= lo and got["ritz"][-1] <= hi
