"""The moments Gram kind on the GPU against the oracle.

No kernel forms P^T A P, nor even P^T M P.  While the basis kernels form p_i,
they sum d_i = <p_i, M p_i> and e_i = <p_i, M p_{i-1}> per block (two
products per column, no extra memory traffic).  The FGS kernel turns the
2s + 1 totals into the moments mu_k of the Chebyshev basis, then into H =
P^T M P by the product rule of Chebyshev polynomials, then into P^T (A P) by
the recurrence (Sec. 2, Definition).  The oracle forms P^T (A P) directly.
These tests check the chain end to end:
- lockstep outer iterations on every operator kind, each basis column within
  1e-12 of the oracle's and G, ctil, atil, x_{k+1} within 1e-10;
- with and without Jacobi, widths 1 to 31;
- two basis steps per launch and one;
- solves to 1e-8 (FP64 only: the kind is refused in FP32+IR).
The CPU tests (test_moments_gram.py) pin the same arithmetic against the
oracle's G without the GPU."""
import numpy as np
import pytest
import torch

import gen
import oracle
from helpers import make_operator, oracle_rhs, ragged_poisson, rel
from test_gpu_gram_rec import CASES as REC_CASES, _oracle_kw

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def t64(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def host(t):
    return t.detach().cpu().numpy()


# the recurrence kind's cases that the moments kind takes (not p_0 = r with
# Jacobi, not the monomial basis), and odd widths on the two-step path
CASES = {k: v for k, v in REC_CASES.items() if k not in ("faces_p0_mode1", "poisson27_monomial_s6")}
CASES["poisson_s7_pairs_and_step"] = (lambda: gen.small_poisson3d(58, 31, 19, seed=21), "stencil", 7, 20, {})
CASES["poisson_s16_one_step"] = (lambda: ragged_poisson(1), "stencil", 16, 25, {"basis_steps": 1})
CASES["poisson_no_precond_s9"] = (lambda: gen.small_poisson3d(30, 20, 10, seed=22), "stencil", 9, 20,
                                  {"precond": False})


@pytest.mark.parametrize("name", list(CASES))
def test_moments_lockstep_fp64(hip, name):
    make, form, s, nu, extra = CASES[name]
    pr = make()
    A, b = oracle_rhs(pr)
    bt = t64(b)
    x = np.zeros(pr.n)
    okw = _oracle_kw(extra)
    with hip.Solver(make_operator(hip, pr, form), s, nu, pr.lmin, pr.lmax, gram="moments", **extra) as sv:
        assert sv.gram_kind == "moments"
        for k in range(3):
            g = sv.step(bt, t64(x), want_basis=(k == 0))
            o = oracle.step(A, b, x, s, nu, pr.lmin, pr.lmax, want_basis=(k == 0), **okw)
            assert o["status"] == 0
            for key in ("G", "ctil", "atil"):
                assert rel(g[key], o[key]) <= 1e-10, (k, key, rel(g[key], o[key]))
            if k == 0:
                P = host(g["P"])
                for j in range(s):
                    assert rel(P[j], o["P"][j]) <= 1e-12, j
            x = host(g["x"])
            assert rel(x, o["x"]) <= 1e-10, k


@pytest.mark.parametrize("name", ["poisson_ragged_s16", "faces_stencil_s8", "c1_csr_2d_s8", "poisson27_s20",
                                  "poisson_s7_pairs_and_step"])
def test_moments_solve(hip, name):
    make, form, s, nu, extra = CASES[name]
    pr = make()
    A, b = oracle_rhs(pr)
    ref = oracle.solve(A, b, None, s, nu, pr.lmin, pr.lmax, 1e-8)
    with hip.Solver(make_operator(hip, pr, form), s, nu, pr.lmin, pr.lmax, gram="moments") as sv:
        x, st = sv.solve(t64(b), None, 1e-8)
    assert st.status == 0
    assert np.linalg.norm(b - oracle.spmv(A, host(x))) / np.linalg.norm(b) <= 1e-8
    assert abs(st.outer_iters - ref["iters"]) <= max(1, int(0.05 * ref["iters"])), (st.outer_iters, ref["iters"])


def test_moments_default_and_limits(hip):
    """AUTO picks the moments kind where it applies and the recurrence kind
    for p_0 = r with Jacobi, the monomial basis and FP32+IR; the moments kind
    is refused beyond s = 31 and where it does not apply."""
    pr = gen.small_poisson3d(12, 10, 9, seed=1)
    op = hip.Operator.stencil(12, 10, 9)
    with hip.Solver(op, 8, 5, pr.lmin, pr.lmax) as sv:
        assert sv.gram_kind == "moments"
    with hip.Solver(op, 8, 5, pr.lmin, pr.lmax, p0_mode=1) as sv:
        assert sv.gram_kind == "recurrence"
    with hip.Solver(op, 8, 5, pr.lmin, pr.lmax, p0_mode=1, precond=False) as sv:
        assert sv.gram_kind == "moments"
    with hip.Solver(op, 8, 5, pr.lmin, pr.lmax, basis="monomial") as sv:
        assert sv.gram_kind == "recurrence"
    with hip.Solver(op, 8, 5, pr.lmin, pr.lmax, precision="fp32ir") as sv:
        assert sv.gram_kind == "recurrence"
    for kw in ({"p0_mode": 1}, {"basis": "monomial"}, {"precision": "fp32ir"}):
        with pytest.raises(hip.SStepError) as e:
            hip.Solver(op, 8, 5, pr.lmin, pr.lmax, gram="moments", **kw)
        assert e.value.name == "SSTEP_E_UNSUPPORTED"
    with pytest.raises(hip.SStepError) as e:
        hip.Solver(op, 32, 5, pr.lmin, pr.lmax, gram="moments")
    assert e.value.name == "SSTEP_E_UNSUPPORTED"
