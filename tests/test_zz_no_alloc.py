"""The allocation-free entry point sstep_solve_noalloc, through the C ABI,
against the existing context entry points (sstep_setup + sstep_solve with the
same default Gram schedule, autotuning off): identical iteration counts and
bitwise-identical solutions, two calls in a row on one GPU with the second
on a smaller problem (the static scratch keeps the first call's contents),
and the true residual recomputed by the oracle.  Also the errors: a problem
beyond the scratch, FP32+IR, host operator arrays, malformed CSR patterns
(checked on the device; every index the check reads is in bounds)."""
import ctypes as C

import numpy as np
import pytest
import torch

import gen
import oracle
from helpers import make_operator, oracle_rhs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def t64(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def dev_operator(hip, pr, form):
    """Library operator with every array in device memory."""
    if form == "csr":
        rp, ci, v = pr.csr()
        return hip.Operator.csr(torch.as_tensor(rp, device=DEV), torch.as_tensor(ci, device=DEV), t64(v))
    if getattr(pr, "stencil", 7) == 27:
        return hip.Operator.stencil27(*pr.dims)
    if pr.kx is None:
        return hip.Operator.stencil(*pr.dims)
    return hip.Operator.stencil(*pr.dims, t64(pr.kx), t64(pr.ky), t64(pr.kz))


def noalloc(hip, op, s, nu, lmin, lmax, b, x, tol=1e-8, precision=0):
    N = hip._native
    lib = N.load()
    opt = N.Options()
    lib.sstep_default_options(C.byref(opt))
    opt.precision = precision
    opt.stream = torch.cuda.current_stream().cuda_stream
    cop = op.to_c()
    st = N.Stats()
    code = lib.sstep_solve_noalloc(C.byref(cop), s, nu, lmin, lmax, C.byref(opt), b.data_ptr(), x.data_ptr(), tol,
                                   C.byref(st))
    return code, st, N.last_error(None)


def reference(hip, pr, form, s, nu, b):
    # the allocation-free entry point takes the recurrence Gram kind
    with hip.Solver(make_operator(hip, pr, form), s, nu, pr.lmin, pr.lmax, autotune=False,
                    gram="recurrence") as sv:
        return sv.solve(b, None, 1e-8)


PAIRS = {
    # (first problem, second smaller problem), operator form, s, nu
    "poisson7_s16": ((lambda: gen.small_poisson3d(48, 40, 36, seed=1),
                           lambda: gen.small_poisson3d(21, 17, 13, seed=2)), "stencil", 16, 25),
    "faces7_s8": ((lambda: gen.small_faces3d(40, 33, 30, seed=3, sigma=1.0),
                         lambda: gen.small_faces3d(17, 11, 9, seed=4, sigma=0.5)), "stencil", 8, 25),
    "csr2d_s8": ((lambda: gen.config1(0),
                         lambda: gen.Problem("p2d", "csr", (20, 13), 8, 20, *gen.jacobi_poisson_bounds(20, 13),
                                             xstar=gen.uniform(gen.rng(5), 260))), "csr", 8, 20),
    "poisson27_s20": ((lambda: gen.small_poisson27(30, 28, 26, seed=6),
                             lambda: gen.small_poisson27(9, 8, 7, seed=7)), "stencil", 20, 30),
}


@pytest.mark.parametrize("name", list(PAIRS))
def test_noalloc_matches_context_solve_twice(hip, name):
    (first, second), form, s, nu = PAIRS[name]
    for make in (first, second):
        pr = make()
        A, b = oracle_rhs(pr)
        bt = t64(b)
        xr, sr = reference(hip, pr, form, s, nu, bt)
        x = torch.zeros_like(bt)
        code, st, msg = noalloc(hip, dev_operator(hip, pr, form), s, nu, pr.lmin, pr.lmax, bt, x)
        torch.cuda.synchronize()
        assert code == 0, msg
        assert st.status == 0 and st.outer_iters == sr.outer_iters, (st.outer_iters, sr.outer_iters)
        assert st.rel_res == sr.rel_res
        assert torch.equal(x, xr), (name, pr.dims)
        assert np.linalg.norm(b - oracle.spmv(A, x.cpu().numpy())) / np.linalg.norm(b) <= 1e-8


def test_noalloc_errors(hip):
    N = hip._native
    pr = gen.small_poisson3d(12, 10, 9)
    A, b = oracle_rhs(pr)
    bt = t64(b)
    x = torch.zeros_like(bt)
    # FP32+IR is not offered
    code, _, msg = noalloc(hip, hip.Operator.stencil(12, 10, 9), 8, 20, pr.lmin, pr.lmax, bt, x, precision=1)
    assert N.STATUS_NAMES[code] == "SSTEP_E_UNSUPPORTED", msg
    # beyond the static scratch: 27-point 200^3 at s = 32 needs ~4 GB
    big = torch.zeros(8, dtype=torch.float64, device=DEV)
    code, _, msg = noalloc(hip, hip.Operator.stencil27(200, 200, 200), 32, 20, 0.001, 1.5, big, big)
    assert N.STATUS_NAMES[code] == "SSTEP_E_ARG" and "too large" in msg, msg
    # host arrays for a CSR operator
    pc = gen.config1(0)
    rp, ci, v = pc.csr()
    bc = t64(oracle.spmv(pc.csr(), pc.xstar))
    xc = torch.zeros_like(bc)
    code, _, msg = noalloc(hip, hip.Operator.csr(rp, ci, v), 8, 20, pc.lmin, pc.lmax, bc, xc)
    assert N.STATUS_NAMES[code] == "SSTEP_E_ARG" and "device memory" in msg, msg
    # malformed patterns, detected on the device before any solve kernel runs
    bad_ci = ci.copy()
    bad_ci[5] = rp.size + 3  # column out of range (rows are well formed)
    code, _, msg = noalloc(hip, hip.Operator.csr(torch.as_tensor(rp, device=DEV), torch.as_tensor(bad_ci, device=DEV),
                                                 t64(v)), 8, 20, pc.lmin, pc.lmax, bc, xc)
    assert N.STATUS_NAMES[code] == "SSTEP_E_ARG" and "malformed" in msg, msg
    bad_rp = rp.copy()
    bad_rp[7], bad_rp[8] = bad_rp[8], bad_rp[7]  # row pointers not monotone
    code, _, msg = noalloc(hip, hip.Operator.csr(torch.as_tensor(bad_rp, device=DEV), torch.as_tensor(ci, device=DEV),
                                                 t64(v)), 8, 20, pc.lmin, pc.lmax, bc, xc)
    assert N.STATUS_NAMES[code] == "SSTEP_E_ARG" and "malformed" in msg, msg
    # after the errors a valid call still works
    code, st, msg = noalloc(hip, hip.Operator.stencil(12, 10, 9), 8, 20, pr.lmin, pr.lmax, bt, x)
    assert code == 0 and st.status == 0, msg
