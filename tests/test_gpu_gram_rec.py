"""The recurrence Gram kind on the GPU against the oracle.

G_raw = P^T (A P) is formed without applying A in the Gram kernel: the basis
keeps p_s, the kernel forms the M-weighted Gram H = P^T M P of p_0 .. p_s, and
the Chebyshev recurrence (Sec. 2, Definition) maps H onto P^T (A P).  The
oracle forms P^T (A P) directly, so these tests check the identity end to
end: lockstep outer iterations (G, ctil, atil, x_{k+1} within 1e-10 entry by
entry) on every operator kind, with and without the Jacobi preconditioner,
both p_0 readings, the monomial basis, s from 1 to 31, and the full 224^3
problem; solves to 1e-8 in FP64 and FP32+IR."""
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
    # name: (problem, form, s, nu, extra solver/oracle options)
    "poisson_ragged_s16": (lambda: ragged_poisson(0), "stencil", 16, 25, {}),
    "faces_stencil_s8": (lambda: gen.small_faces3d(23, 17, 13, seed=2, sigma=1.0), "stencil", 8, 25, {}),
    "faces_csr_s5": (lambda: gen.small_faces3d(19, 21, 7, seed=3, sigma=0.5), "csr", 5, 20, {}),
    "c1_csr_2d_s8": (lambda: gen.config1(0), "csr", 8, 20, {}),
    "poisson27_s20": (lambda: gen.small_poisson27(19, 21, 9, seed=2), "stencil", 20, 30, {}),
    "poisson_s1": (lambda: gen.small_poisson3d(9, 8, 7, seed=5), "stencil", 1, 3, {}),
    "poisson_s31": (lambda: gen.small_poisson3d(20, 18, 16, seed=4), "stencil", 31, 30, {}),
    # widths at the kernel's column-block boundaries: 16 basis columns (s = 15),
    # 17 (s = 16, one column beside the matrix-core block), 18 (s = 17, the
    # second block's first width), 25 (s = 24) with a varying diagonal on CSR
    "poisson_s15": (lambda: gen.small_poisson3d(13, 11, 9, seed=12), "stencil", 15, 20, {}),
    "faces_stencil_s17": (lambda: gen.small_faces3d(17, 13, 11, seed=13, sigma=1.0), "stencil", 17, 25, {}),
    "faces_csr_s24": (lambda: gen.small_faces3d(14, 15, 9, seed=14, sigma=0.5), "csr", 24, 30, {}),
    "faces_no_precond": (lambda: gen.small_faces3d(15, 13, 11, seed=7, sigma=0.5), "stencil", 6, 20,
                         {"precond": False}),
    "faces_p0_mode1": (lambda: gen.small_faces3d(15, 13, 11, seed=8, sigma=1.0), "stencil", 8, 20, {"p0_mode": 1}),
    "poisson27_monomial_s6": (lambda: gen.small_poisson27(16, 13, 11, seed=11), "stencil", 6, 20,
                              {"basis": "monomial"}),
}


def _oracle_kw(extra):
    kw = {}
    if "precond" in extra:
        kw["precond"] = 1 if extra["precond"] else 0
    if "p0_mode" in extra:
        kw["p0_mode"] = extra["p0_mode"]
    if "basis" in extra:
        kw["basis"] = extra["basis"]
    return kw


@pytest.mark.parametrize("name", list(CASES))
def test_recurrence_lockstep_fp64(hip, name):
    make, form, s, nu, extra = CASES[name]
    pr = make()
    A, b = oracle_rhs(pr)
    bt = t64(b)
    x = np.zeros(pr.n)
    okw = _oracle_kw(extra)
    with hip.Solver(make_operator(hip, pr, form), s, nu, pr.lmin, pr.lmax, gram="recurrence", **extra) as sv:
        assert sv.gram_kind == "recurrence"
        for k in range(3):
            g = sv.step(bt, t64(x), want_basis=(k == 0))
            o = oracle.step(A, b, x, s, nu, pr.lmin, pr.lmax, want_basis=(k == 0), **okw)
            assert o["status"] == 0
            for key in ("G", "ctil", "atil"):
                assert rel(g[key], o[key]) <= 1e-10, (k, key, rel(g[key], o[key]))
            if k == 0:
                P, AP = host(g["P"]), host(g["AP"])
                for j in range(s):
                    assert rel(P[j], o["P"][j]) <= 1e-12 and rel(AP[j], o["AP"][j]) <= 1e-12, j
            x = host(g["x"])
            assert rel(x, o["x"]) <= 1e-10, k


@pytest.mark.parametrize("name", ["poisson_ragged_s16", "faces_stencil_s8", "c1_csr_2d_s8", "poisson27_s20"])
@pytest.mark.parametrize("precision", ["fp64", "fp32ir"])
def test_recurrence_solve(hip, name, precision):
    make, form, s, nu, extra = CASES[name]
    pr = make()
    A, b = oracle_rhs(pr)
    ref = oracle.solve(A, b, None, s, nu, pr.lmin, pr.lmax, 1e-8)
    with hip.Solver(make_operator(hip, pr, form), s, nu, pr.lmin, pr.lmax, gram="recurrence",
                    precision=precision) as sv:
        x, st = sv.solve(t64(b), None, 1e-8)
    assert st.status == 0
    assert np.linalg.norm(b - oracle.spmv(A, host(x))) / np.linalg.norm(b) <= 1e-8
    if precision == "fp64":
        assert abs(st.outer_iters - ref["iters"]) <= max(1, int(0.05 * ref["iters"])), (st.outer_iters, ref["iters"])


def test_recurrence_width_limit(hip):
    pr = gen.small_poisson3d(10, 9, 8)
    with pytest.raises(hip.SStepError) as e:
        hip.Solver(hip.Operator.stencil(10, 9, 8), 32, 20, pr.lmin, pr.lmax, gram="recurrence")
    assert e.value.name == "SSTEP_E_UNSUPPORTED"


def test_recurrence_full_size_224(hip):
    """The 224^3 problem with the recurrence kind, autotuned schedule: two
    lockstep outer iterations against the oracle and the solve to 1e-8."""
    N, S, NU = 224, 16, 25
    pr = gen.config2(0, N=N, s=S, nu=NU)
    A = oracle.assemble_stencil7(N, N, N)
    b = oracle.spmv(A, pr.xstar)
    bt = t64(b)
    x = np.zeros(pr.n)
    with hip.Solver(hip.Operator.stencil(N, N, N), S, NU, pr.lmin, pr.lmax, gram="recurrence") as sv:
        for k in range(2):
            g = sv.step(bt, t64(x))
            o = oracle.step(A, b, x, S, NU, pr.lmin, pr.lmax)
            for key in ("G", "ctil", "atil"):
                assert rel(g[key], o[key]) <= 1e-10, (k, key, rel(g[key], o[key]))
            x = host(g["x"])
            assert rel(x, o["x"]) <= 1e-10, k
        xs, st = sv.solve(bt, None, 1e-8)
    assert st.status == 0
    assert np.linalg.norm(b - oracle.spmv(A, host(xs))) / np.linalg.norm(b) <= 1e-8
