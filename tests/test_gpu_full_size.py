"""The headline workload at its full size: 224^3 Poisson (11,239,424 unknowns),
s = 16, nu = 25, matrix-free stencil, FP64, with the solver built exactly as
the benchmark builds it (default options, so the recurrence Gram kind, the
autotuned schedule and the graph-chunked solve).

Two checks against the oracle:
- lockstep: two outer iterations from the same x_k, each compared with the
  oracle's outer iteration (a few seconds each on the host): G, ctil, atil and
  x_{k+1} within 1e-10 relative both norm-wise and entry by entry (every
  |difference| within 1e-10 of the vector's largest entry), ||r_k|| within
  1e-12, and the Gram diagnostics delta_k and ||L||_F;
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
        assert sv.gram_kind == "moments"
        for k in range(2):
            g = sv.step(bt, t64(x))
            o = oracle.step(A, b, x, S, NU, pr.lmin, pr.lmax)
            assert o["status"] == 0
            assert abs(g["rnorm"] - o["rnorm"]) <= 1e-12 * o["rnorm"], k
            for key in ("G", "ctil", "atil"):
                assert rel(g[key], o[key]) <= 1e-10, (k, key, rel(g[key], o[key]))
            d = sv.last_iteration()
            assert abs(d["lnorm"] - o["lnorm"]) <= 1e-10 * o["lnorm"], (k, d["lnorm"], o["lnorm"])
            assert abs(d["delta"] - o["delta"]) <= 1e-8 * o["delta"], (k, d["delta"], o["delta"])
            x = host(g["x"])
            assert rel(x, o["x"]) <= 1e-10, k


def test_full_size_solve_follows_oracle(hip, c2):
    pr, A, b = c2
    with open(GOLDEN) as f:
        ref = json.load(f)
    assert ref["status"] == 0
    with hip.Solver(hip.Operator.stencil(N, N, N), S, NU, pr.lmin, pr.lmax, record_history=True) as sv:
        assert sv.gram_kind == "moments"
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


@pytest.mark.parametrize("s,nu", gen.config3_sweep())
@pytest.mark.parametrize("precision", ["fp64", "fp32ir"])
def test_full_size_c3_sweep_pair(hip, c2, s, nu, precision):
    """The mixed-precision sweep at the 224^3 problem's full size, every
    (s, nu) pair in both precisions, with the solver built as the benchmark
    builds it (default Gram kind and autotuned schedule for the pair): the
    true relative residual, recomputed by the oracle in FP64, reaches 1e-8.
    For FP32+IR the FP32 inner error of the first outer iteration is measured
    against the oracle's FP64 step from the same x_0 = 0 (lockstep):
    ||dx32 - dx64|| / ||dx64|| and ||G32 - G64|| / ||G64|| (reported, and
    bounded by 1e-4 as a sanity gate)."""
    pr, A, b = c2
    bt = t64(b)
    with hip.Solver(hip.Operator.stencil(N, N, N), s, nu, pr.lmin, pr.lmax, precision=precision) as sv:
        x, st = sv.solve(bt, None, 1e-8)
        assert st.status == 0
        true_rel = np.linalg.norm(b - oracle.spmv(A, host(x))) / np.linalg.norm(b)
        assert true_rel <= 1e-8, (s, nu, precision, true_rel)
        if precision == "fp32ir":
            g = sv.step(bt, t64(np.zeros(pr.n)))
            o = oracle.step(A, b, np.zeros(pr.n), s, nu, pr.lmin, pr.lmax)
            dx = np.linalg.norm(host(g["x"]) - o["x"]) / np.linalg.norm(o["x"])
            dG = np.linalg.norm(g["G"] - o["G"]) / np.linalg.norm(o["G"])
            print(f"s={s} nu={nu}: {st.outer_iters} outer, FP32 inner error dx {dx:.2e}, G {dG:.2e}")
            assert dx <= 1e-4 and dG <= 1e-4, (dx, dG)
        else:
            print(f"s={s} nu={nu}: {st.outer_iters} outer (FP64)")


C5_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_oracle_grad.json")


def test_full_size_c5_gradient_matches_oracle(hip):
    """The differentiable solve at its full size (128^3 faces, sigma 0.5):
    the autograd gradient (forward and adjoint at tol 1e-12) against the
    oracle's reference gradient (tests/golden/c5_oracle_grad.json, written by
    tests/golden/make_golden.py --c5 from the oracle alone), entry by entry at
    the fixture's sampled positions and through the full vectors' norms; the
    error at the benchmark tolerance 1e-8 is reported."""
    with open(C5_GOLDEN) as f:
        ref = json.load(f)
    assert ref["status"] == [0, 0]
    pr = gen.config5(0)
    nx, ny, nz = pr.dims
    ik, iv = np.asarray(ref["idx_k"]), np.asarray(ref["idx_v"])
    op = hip.Operator.stencil(nx, ny, nz, pr.kx, pr.ky, pr.kz)
    errs = {}
    with hip.Solver(op, pr.s, pr.nu, pr.lmin, pr.lmax) as sv:
        for tol in (1e-12, 1e-8):
            coeffs = t64(np.concatenate([pr.kx, pr.ky, pr.kz])).requires_grad_(True)
            bt = t64(pr.rhs[0]).requires_grad_(True)
            x = hip.sstep_solve(coeffs, bt, sv, tol)
            (0.5 * torch.sum((x - t64(pr.xtarget)) ** 2)).backward()
            gk, gb, xh = host(coeffs.grad), host(bt.grad), host(x)
            errs[tol] = dict(x=rel(xh[iv], ref["x"]), lam=rel(gb[iv], ref["lam"]), dk=rel(gk[ik], ref["dk"]),
                             norm_dk=abs(np.linalg.norm(gk) - ref["norm_dk"]) / ref["norm_dk"],
                             norm_lam=abs(np.linalg.norm(gb) - ref["norm_lam"]) / ref["norm_lam"])
    print(f"128^3 gradient vs oracle: tol 1e-12 {errs[1e-12]}; tol 1e-8 {errs[1e-8]}")
    e = errs[1e-12]
    assert e["x"] <= 1e-8 and e["lam"] <= 1e-7 and e["dk"] <= 1e-7, e
    assert e["norm_dk"] <= 1e-8 and e["norm_lam"] <= 1e-8, e
    assert errs[1e-8]["dk"] <= 1e-3, errs[1e-8]
