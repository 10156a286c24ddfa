"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: per outer iteration, the scaled FGS solution atil and the new
iterate x_{k+1} agree with the oracle to 1e-10 relative in FP64 mode when both
start from the same x_k (lockstep); free-running solves reach a final relative
residual <= 1e-8 recomputed by the oracle in FP64, in every mode.
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
    # name: (problem factory, operator form, s, nu)
    "c1_csr_2d": (lambda: gen.config1(0), "csr", 8, 20),
    "poisson_ragged_stencil": (lambda: ragged_poisson(0), "stencil", 16, 25),
    "poisson_ragged_csr": (lambda: ragged_poisson(1), "csr", 16, 25),
    "faces_stencil_s8": (lambda: gen.small_faces3d(23, 17, 13, seed=2, sigma=1.0), "stencil", 8, 25),
    "faces_csr_s5": (lambda: gen.small_faces3d(19, 21, 7, seed=3, sigma=0.5), "csr", 5, 20),
    "poisson_s32": (lambda: gen.small_poisson3d(20, 18, 16, seed=4), "stencil", 32, 30),
    "poisson_s1": (lambda: gen.small_poisson3d(9, 8, 7, seed=5), "stencil", 1, 3),
}


@pytest.mark.parametrize("name", list(CASES))
def test_apply_matches_oracle(hip, name):
    make, form, s, nu = CASES[name]
    pr = make()
    A = oracle.problem_csr(pr)
    x = gen.uniform(gen.rng(99), pr.n)
    want = oracle.spmv(A, x)
    with hip.Solver(make_operator(hip, pr, form), s, nu, pr.lmin, pr.lmax) as sv:
        got = host(sv.apply(t64(x)))
    rp, ci, v = A
    absA = np.abs(v)
    scale = np.add.reduceat(absA * np.abs(x[ci]), rp[:-1])
    assert np.all(np.abs(got - want) <= 1e-14 * scale + 1e-300)


@pytest.mark.parametrize("name", list(CASES))
def test_lockstep_outer_iterations_fp64(hip, name):
    """atil, G, ctil, x_{k+1} of each outer iteration from the same x_k."""
    make, form, s, nu = CASES[name]
    pr = make()
    A, b = oracle_rhs(pr)
    bt = t64(b)
    x = np.zeros(pr.n)
    with hip.Solver(make_operator(hip, pr, form), s, nu, pr.lmin, pr.lmax) as sv:
        for k in range(4):
            xt = t64(x)
            g = sv.step(bt, xt, want_basis=(k == 0))
            o = oracle.step(A, b, x, s, nu, pr.lmin, pr.lmax, want_basis=(k == 0))
            assert o["status"] == 0
            assert abs(g["rnorm"] - o["rnorm"]) <= 1e-12 * o["rnorm"], k
            assert rel(g["G"], o["G"]) <= 1e-10, k
            assert rel(g["ctil"], o["ctil"]) <= 1e-10, k
            assert rel(g["atil"], o["atil"]) <= 1e-10, (k, rel(g["atil"], o["atil"]))
            xn = host(g["x"])
            assert rel(xn, o["x"]) <= 1e-10, k
            # Gram diagnostics of the same iteration (Sec. 7 delta, Sec. 4 ||L||_F)
            d = sv.last_iteration()
            assert abs(d["rnorm"] - o["rnorm"]) <= 1e-12 * o["rnorm"], k
            assert abs(d["lnorm"] - o["lnorm"]) <= 1e-10 * o["lnorm"], (k, d["lnorm"], o["lnorm"])
            assert abs(d["delta"] - o["delta"]) <= 1e-8 * o["delta"] + 1e-14, (k, d["delta"], o["delta"])
            if k == 0:
                P, AP = host(g["P"]), host(g["AP"])
                for j in range(s):
                    assert rel(P[j], o["P"][j]) <= 1e-12, ("P", j)
                    assert rel(AP[j], o["AP"][j]) <= 1e-12, ("AP", j)
            x = xn


@pytest.mark.parametrize("name", ["c1_csr_2d", "poisson_ragged_stencil", "faces_stencil_s8", "faces_csr_s5"])
@pytest.mark.parametrize("chunk", [1, 4])
def test_free_running_solve_fp64(hip, name, chunk):
    make, form, s, nu = CASES[name]
    pr = make()
    A, b = oracle_rhs(pr)
    ref = oracle.solve(A, b, None, s, nu, pr.lmin, pr.lmax, 1e-8, hist_cap=2000)
    assert ref["status"] == 0
    with hip.Solver(make_operator(hip, pr, form), s, nu, pr.lmin, pr.lmax, graph_chunk=chunk,
                    record_history=True) as sv:
        x, st = sv.solve(t64(b), None, 1e-8, history=True)
    # per-update Gram diagnostics follow the oracle's while the trajectories
    # agree (the first three updates)
    assert st.hist_delta.shape == st.hist_lnorm.shape == (st.outer_iters,)
    for k in range(3):
        assert abs(st.hist_lnorm[k] - ref["hist_lnorm"][k]) <= 1e-9 * ref["hist_lnorm"][k], k
        assert abs(st.hist_delta[k] - ref["hist_delta"][k]) <= 1e-7 * ref["hist_delta"][k] + 1e-14, k
    assert np.all(st.hist_delta > 0) and np.all(st.hist_lnorm > 0)
    xh = host(x)
    true_rel = np.linalg.norm(b - oracle.spmv(A, xh)) / np.linalg.norm(b)
    assert true_rel <= 1e-8
    assert abs(st.outer_iters - ref["iters"]) <= max(1, int(0.05 * ref["iters"]))
    assert abs(st.rel_res - true_rel) <= 1e-12
    assert st.hist_relres.shape == (st.outer_iters + 1,)
    assert st.hist_relres[0] == 1.0 and st.hist_relres[-1] < 1e-8
    # the first three iterates follow the oracle's free-running trajectory
    x = np.zeros(pr.n)
    xg = t64(x)
    with hip.Solver(make_operator(hip, pr, form), s, nu, pr.lmin, pr.lmax) as sv:
        for k in range(3):
            sv.step(t64(b), xg)
            x = oracle.step(A, b, x, s, nu, pr.lmin, pr.lmax)["x"]
            assert rel(host(xg), x) <= 1e-10, k


def test_solve_is_bitwise_reproducible(hip):
    pr = ragged_poisson(3)
    A, b = oracle_rhs(pr)
    with hip.Solver(make_operator(hip, pr, "stencil"), 16, 25, pr.lmin, pr.lmax) as sv:
        x1, s1 = sv.solve(t64(b))
        x2, s2 = sv.solve(t64(b))
    assert s1.outer_iters == s2.outer_iters
    assert torch.equal(x1, x2)


def test_graph_chunks_give_identical_results(hip):
    pr = gen.small_faces3d(15, 14, 13, seed=6)
    A, b = oracle_rhs(pr)
    res = []
    for chunk in (1, 3, 8):
        with hip.Solver(make_operator(hip, pr, "stencil"), 8, 25, pr.lmin, pr.lmax, graph_chunk=chunk) as sv:
            res.append(sv.solve(t64(b)))
    for x, st in res[1:]:
        assert st.outer_iters == res[0][1].outer_iters
        assert torch.equal(x, res[0][0])


def test_nonzero_initial_guess_and_p0_mode(hip):
    pr = gen.small_faces3d(12, 11, 10, seed=7)
    A, b = oracle_rhs(pr)
    x0 = 0.5 * gen.uniform(gen.rng(1), pr.n)
    for p0_mode in (0, 1):
        ref = oracle.solve(A, b, x0, 6, 20, pr.lmin, pr.lmax, 1e-9, p0_mode=p0_mode)
        with hip.Solver(make_operator(hip, pr, "stencil"), 6, 20, pr.lmin, pr.lmax, p0_mode=p0_mode) as sv:
            x, st = sv.solve(t64(b), t64(x0), 1e-9)
        assert abs(st.outer_iters - ref["iters"]) <= max(1, int(0.05 * ref["iters"]))
        assert np.linalg.norm(b - oracle.spmv(A, host(x))) <= 1e-9 * np.linalg.norm(b - oracle.spmv(A, x0))


def test_no_preconditioner(hip):
    pr = gen.small_poisson3d(10, 9, 8, seed=8)
    A, b = oracle_rhs(pr)
    lmin, lmax = 6 * pr.lmin, 6 * pr.lmax  # spectrum of A itself
    ref = oracle.solve(A, b, None, 6, 20, lmin, lmax, 1e-8, precond=0)
    with hip.Solver(make_operator(hip, pr, "stencil"), 6, 20, lmin, lmax, precond=False) as sv:
        x, st = sv.solve(t64(b))
        g = sv.step(t64(b), torch.zeros(pr.n, dtype=torch.float64, device=DEV))
    o = oracle.step(A, b, np.zeros(pr.n), 6, 20, lmin, lmax, precond=0)
    assert rel(g["atil"], o["atil"]) <= 1e-10
    assert abs(st.outer_iters - ref["iters"]) <= max(1, int(0.05 * ref["iters"]))


# ---------------------------------------------------------------------------
# edge cases and failure paths
# ---------------------------------------------------------------------------

def test_zero_rhs_returns_immediately(hip):
    pr = gen.small_poisson3d(8, 8, 8)
    with hip.Solver(make_operator(hip, pr, "stencil"), 4, 5, pr.lmin, pr.lmax) as sv:
        x, st = sv.solve(torch.zeros(pr.n, dtype=torch.float64, device=DEV))
    assert st.outer_iters == 0 and st.status == 0 and torch.all(x == 0)


def test_single_unknown_grid(hip):
    # 1x1x1 grid: A = [6], one outer iteration solves it exactly
    with hip.Solver(hip.Operator.stencil(1, 1, 1), 1, 1, 0.5, 1.5) as sv:
        x, st = sv.solve(t64([3.0]))
    assert abs(host(x)[0] - 0.5) < 1e-15 and st.outer_iters == 1


def test_nonfinite_rhs(hip):
    pr = gen.small_poisson3d(8, 8, 8)
    b = np.ones(pr.n)
    b[17] = np.nan
    with hip.Solver(make_operator(hip, pr, "stencil"), 4, 5, pr.lmin, pr.lmax) as sv:
        with pytest.raises(hip.SStepError) as ei:
            sv.solve(t64(b))
    assert ei.value.name == "SSTEP_E_NONFINITE"


def test_breakdown_when_basis_vector_vanishes(hip):
    n = 100
    rp = np.arange(n + 1, dtype=np.int32)
    op = hip.Operator.csr(rp, np.arange(n, dtype=np.int32), np.full(n, 2.0))
    with hip.Solver(op, 3, 5, 1.0, 3.0, precond=False) as sv:
        with pytest.raises(hip.SStepError) as ei:
            sv.solve(t64(np.ones(n)))
    assert ei.value.name == "SSTEP_E_BREAKDOWN"
    assert ei.value.stats.outer_iters == 0


def test_max_outer_gives_noconv_and_last_iterate(hip):
    pr = gen.config1(0)
    A, b = oracle_rhs(pr)
    ref = oracle.solve(A, b, None, pr.s, pr.nu, pr.lmin, pr.lmax, 1e-8, max_outer=5)
    assert ref["status"] == 5
    with hip.Solver(make_operator(hip, pr, "csr"), pr.s, pr.nu, pr.lmin, pr.lmax, max_outer=5) as sv:
        x, st = sv.solve(t64(b), None, 1e-8, raise_on_error=False)
    assert st.status == 5 and st.outer_iters == 5
    assert rel(host(x), ref["x"]) <= 1e-9


def test_update_coefficients_changes_operator(hip):
    pr = gen.small_faces3d(9, 8, 7, seed=9)
    pr2 = gen.small_faces3d(9, 8, 7, seed=10)
    A2, b = oracle_rhs(pr2)
    with hip.Solver(make_operator(hip, pr, "stencil"), 6, 20, 0.0, 2.0) as sv:
        sv.update_coefficients(make_operator(hip, pr2, "stencil"))
        x, st = sv.solve(t64(b))
    assert np.linalg.norm(b - oracle.spmv(A2, host(x))) <= 1e-8 * np.linalg.norm(b)


def test_device_resident_operator_arrays(hip):
    pr = gen.small_faces3d(11, 10, 9, seed=11)
    A, b = oracle_rhs(pr)
    rp, ci, v = pr.csr()
    op = hip.Operator.csr(torch.as_tensor(rp, device=DEV), torch.as_tensor(ci, device=DEV), t64(v))
    with hip.Solver(op, 6, 20, pr.lmin, pr.lmax) as sv:
        x, st = sv.solve(t64(b))
    assert np.linalg.norm(b - oracle.spmv(A, host(x))) <= 1e-8 * np.linalg.norm(b)


def test_setup_rejects_negative_diagonal(hip):
    n = 10
    v = np.full(n, 2.0)
    v[4] = -1.0
    op = hip.Operator.csr(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), v)
    with pytest.raises(hip.SStepError) as ei:
        hip.Solver(op, 2, 2, 0.1, 2.0)
    assert ei.value.name == "SSTEP_E_ARG"
