"""The headline workload at its full size: 224^3 Poisson (11,239,424 unknowns),
s = 16, nu = 25, matrix-free stencil, FP64, with the solver built exactly as
the benchmark builds it (default options, so the Gram kernel that applies the
operator itself, the autotuned schedule and the graph-chunked solve).

Two checks against the oracle:
- lockstep: two outer iterations from the same x_k, each compared entry by
  entry with the oracle's outer iteration (a few seconds each on the host),
  G, ctil, atil and x_{k+1} within 1e-10 relative, ||r_k|| within 1e-12;
- free-running: the solve stops within 5% (at least one) of the oracle's
  outer-iteration count for the same problem (tests/golden/c2_oracle.json,
  written by tests/golden/make_golden.py --c2 from the oracle alone), its
  first relative residuals follow the oracle's history, and the true relative
  residual ||b - A x|| / ||b||, recomputed by the oracle, is <= 1e-8.

The same problem in FP32+IR, the 128^3 face-coefficient workload of the
differentiable solve (forward, adjoint, gradient scatter), the batched
workload (64 systems x 8 right-hand sides) and the CSR form of the 224^3
problem are checked at their full sizes too.
"""
import json
import os

import numpy as np
import pytest
import torch

import gen
import oracle
from helpers import rel

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
N, S, NU = 224, 16, 25
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_oracle.json")


def t64(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def c2():
    pr = gen.config2(0, N=N, s=S, nu=NU)
    A = oracle.assemble_stencil7(N, N, N)
    b = oracle.spmv(A, pr.xstar)
    return pr, A, b


def test_full_size_lockstep_matches_oracle(hip, c2):
    pr, A, b = c2
    bt = t64(b)
    x = np.zeros(pr.n)
    with hip.Solver(hip.Operator.stencil(N, N, N), S, NU, pr.lmin, pr.lmax) as sv:
        assert sv.gram_applies_operator
        for k in range(2):
            g = sv.step(bt, t64(x))
            o = oracle.step(A, b, x, S, NU, pr.lmin, pr.lmax)
            assert o["status"] == 0
            assert abs(g["rnorm"] - o["rnorm"]) <= 1e-12 * o["rnorm"], k
            for key in ("G", "ctil", "atil"):
                assert rel(g[key], o[key]) <= 1e-10, (k, key, rel(g[key], o[key]))
            x = host(g["x"])
            assert rel(x, o["x"]) <= 1e-10, k


def test_full_size_solve_follows_oracle(hip, c2):
    pr, A, b = c2
    with open(GOLDEN) as f:
        ref = json.load(f)
    assert ref["status"] == 0
    with hip.Solver(hip.Operator.stencil(N, N, N), S, NU, pr.lmin, pr.lmax, record_history=True) as sv:
        assert sv.gram_applies_operator
        x, st = sv.solve(t64(b), None, 1e-8, history=True)
    assert st.status == 0
    assert abs(st.outer_iters - ref["iters"]) <= max(1, int(0.05 * ref["iters"])), (st.outer_iters, ref["iters"])
    hist = np.asarray(ref["hist_relres"])
    k = min(6, st.outer_iters + 1, hist.size)
    assert np.all(np.abs(st.hist_relres[:k] - hist[:k]) <= 1e-8 * hist[:k]), (st.hist_relres[:k], hist[:k])
    true_rel = np.linalg.norm(b - oracle.spmv(A, host(x))) / np.linalg.norm(b)
    assert true_rel <= 1e-8
    assert abs(st.rel_res - true_rel) <= 1e-12


def test_full_size_fp32ir_reaches_tolerance(hip, c2):
    """The mixed-precision leg of the benchmark at full size: FP64 residual
    and update around an FP32 basis and Gram; the true relative residual,
    recomputed by the oracle in FP64, reaches 1e-8."""
    pr, A, b = c2
    with hip.Solver(hip.Operator.stencil(N, N, N), S, NU, pr.lmin, pr.lmax, precision="fp32ir") as sv:
        x, st = sv.solve(t64(b), None, 1e-8)
    assert st.status == 0
    true_rel = np.linalg.norm(b - oracle.spmv(A, host(x))) / np.linalg.norm(b)
    assert true_rel <= 1e-8


def test_full_size_faces_forward_and_adjoint(hip):
    """The differentiable workload at its full size (128^3 log-normal face
    coefficients, sigma 0.5, s = 16, nu = 25): two lockstep outer iterations
    against the oracle (1e-10), the forward and the adjoint solve to a true
    relative residual <= 1e-8 (recomputed by the oracle), and the face
    gradient scatter bit-identical to the oracle's."""
    pr = gen.config5(0)
    nx, ny, nz = pr.dims
    A = oracle.problem_csr(pr)
    b = pr.rhs[0]
    x = np.zeros(pr.n)
    with hip.Solver(hip.Operator.stencil(nx, ny, nz, pr.kx, pr.ky, pr.kz), pr.s, pr.nu, pr.lmin, pr.lmax) as sv:
        bt = t64(b)
        for k in range(2):
            g = sv.step(bt, t64(x))
            o = oracle.step(A, b, x, pr.s, pr.nu, pr.lmin, pr.lmax)
            assert o["status"] == 0
            for key in ("G", "ctil", "atil"):
                assert rel(g[key], o[key]) <= 1e-10, (k, key, rel(g[key], o[key]))
            x = host(g["x"])
            assert rel(x, o["x"]) <= 1e-10, k
        xs, st = sv.solve(bt, None, 1e-8)
        assert st.status == 0
        xh = host(xs)
        assert np.linalg.norm(b - oracle.spmv(A, xh)) / np.linalg.norm(b) <= 1e-8
        gvec = xh - pr.xtarget
        lam, sta = sv.solve_adjoint(t64(gvec), None, 1e-8)
        assert sta.status == 0
        lh = host(lam)
        assert np.linalg.norm(gvec - oracle.spmv(A, lh)) / np.linalg.norm(gvec) <= 1e-8
        dA = host(sv.grad_operator(lam, xs))
    assert np.array_equal(dA, np.concatenate(oracle.grad_faces(nx, ny, nz, lh, xh)))


@pytest.mark.parametrize("precision", ["fp64", "fp32ir"])
def test_full_size_batched_pairs_reach_tolerance(hip, precision):
    """The batched workload at its full size (64 face-coefficient systems,
    sides U{32..96}, 8 right-hand sides each, s = 16, nu = 25) built as the
    benchmark builds it: every one of the 512 pairs stops with a true relative
    residual <= 1e-8, recomputed by the oracle in FP64, and the reported
    residual matches it."""
    probs = gen.config4(seed=0, nsys=64)
    ops = [hip.Operator.stencil(*p.dims, p.kx, p.ky, p.kz) for p in probs]
    b = [np.concatenate(p.rhs) for p in probs]
    with hip.BatchedSolver(ops, 8, 16, 25, [p.lmin for p in probs], [p.lmax for p in probs],
                           precision=precision) as bs:
        x, st = bs.solve([t64(bq) for bq in b], None, 1e-8)
    assert len(st) == 64 * 8
    worst = 0.0
    for q, p in enumerate(probs):
        A = oracle.problem_csr(p)
        xq = host(x[q])
        for r in range(8):
            sl = slice(r * p.n, (r + 1) * p.n)
            true_rel = np.linalg.norm(b[q][sl] - oracle.spmv(A, xq[sl])) / np.linalg.norm(b[q][sl])
            pst = st[q * 8 + r]
            assert pst.status == 0 and true_rel <= 1e-8, (q, r, pst.status, true_rel)
            assert abs(pst.rel_res - true_rel) <= 1e-10, (q, r, pst.rel_res, true_rel)
            worst = max(worst, true_rel)
    assert worst > 0.0


def test_full_size_csr_matches_oracle(hip, c2):
    """The headline problem given as a CSR matrix (the benchmark's CSR leg):
    one lockstep outer iteration against the oracle (1e-10) and the solve to a
    true relative residual <= 1e-8."""
    pr, A, b = c2
    rp, ci, v = gen.poisson3d_csr(N, N, N)
    with hip.Solver(hip.Operator.csr(rp, ci, v), S, NU, pr.lmin, pr.lmax) as sv:
        assert not sv.gram_applies_operator
        bt = t64(b)
        g = sv.step(bt, t64(np.zeros(pr.n)))
        o = oracle.step(A, b, np.zeros(pr.n), S, NU, pr.lmin, pr.lmax)
        for key in ("G", "ctil", "atil"):
            assert rel(g[key], o[key]) <= 1e-10, (key, rel(g[key], o[key]))
        assert rel(host(g["x"]), o["x"]) <= 1e-10
        x, st = sv.solve(bt, None, 1e-8)
    assert st.status == 0
    assert np.linalg.norm(b - oracle.spmv(A, host(x))) / np.linalg.norm(b) <= 1e-8
