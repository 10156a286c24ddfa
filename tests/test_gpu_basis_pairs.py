"""Two basis steps per launch for the constant 7-point operator, on the GPU
against the oracle.

One launch forms p_{j+1} and p_{j+2} from p_{j-1} and p_j (the Chebyshev
recurrence of Sec. 2, Definition, taken twice): in-plane tiles overlap by a
one-point ring, and each block marches a range of z-planes, reading two planes
below the range and one above it.  The grids here are ragged against the tile
shape in x and y.  They are small enough that the ranges are 4 planes thick,
so most blocks have ranges above and below them.  The cases cover:
- even and odd column counts (an odd count ends with a single step);
- the Gram kinds that keep no AP (moments, the default; recurrence;
  operator-applying);
- Jacobi on and off, and both p_0 readings;
- widths from 2 to 31, and FP32.
The bar for FP64 is the lockstep bar of the single-step path: every basis
column within 1e-12 of the oracle's; G, ctil, atil and x_{k+1} within 1e-10."""
import numpy as np
import pytest
import torch

import gen
import oracle
from helpers import make_operator, oracle_rhs, rel

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def t64(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def host(t):
    return t.detach().cpu().numpy()


CASES = {
    # name: (grid, s, nu, solver options); m = s columns (recurrence kind) or
    # s - 1 (operator-applying kind)
    "rec_s16_ragged": ((61, 47, 23), 16, 25, {}),
    "rec_s7_odd": ((58, 31, 19), 7, 20, {}),
    "apply_s16_odd": ((57, 29, 21), 16, 25, {"gram": "apply"}),
    "apply_s9_even": ((120, 15, 9), 9, 20, {"gram": "apply"}),
    "rec_s2_first_pair_only": ((33, 33, 33), 2, 5, {}),
    "rec_s1_single_step": ((20, 9, 7), 1, 3, {}),
    "rec_s3_no_precond": ((40, 17, 13), 3, 10, {"precond": False}),
    "rec_s8_p0_mode1": ((64, 14, 30), 8, 20, {"p0_mode": 1}),
    "rec_s31": ((24, 20, 18), 31, 30, {}),
    "rec_s12_thin_z": ((70, 45, 3), 12, 20, {}),
    # the default Gram kind is the moments kind; these two take the
    # recurrence kind, whose Gram kernel reads the columns back
    "recurrence_kind_s16": ((61, 47, 23), 16, 25, {"gram": "recurrence"}),
    "recurrence_kind_s7_odd": ((58, 31, 19), 7, 20, {"gram": "recurrence"}),
}


def _oracle_kw(extra):
    kw = {}
    if "precond" in extra:
        kw["precond"] = 1 if extra["precond"] else 0
    if "p0_mode" in extra:
        kw["p0_mode"] = extra["p0_mode"]
    return kw


@pytest.mark.parametrize("name", list(CASES))
def test_pairs_lockstep_fp64(hip, name):
    (nx, ny, nz), s, nu, extra = CASES[name]
    pr = gen.small_poisson3d(nx, ny, nz, seed=len(name))
    A, b = oracle_rhs(pr)
    bt = t64(b)
    x = np.zeros(pr.n)
    okw = _oracle_kw(extra)
    m = s - 1 if extra.get("gram") == "apply" else s
    with hip.Solver(hip.Operator.stencil(nx, ny, nz), s, nu, pr.lmin, pr.lmax, **extra) as sv:
        assert sv.basis_pairs == m // 2, (sv.basis_pairs, m)
        assert sv.basis_launches == m // 2 + m % 2
        for k in range(3):
            g = sv.step(bt, t64(x), want_basis=(k == 0))
            o = oracle.step(A, b, x, s, nu, pr.lmin, pr.lmax, want_basis=(k == 0), **okw)
            assert o["status"] == 0
            if k == 0:
                P = host(g["P"])
                for j in range(s):
                    assert rel(P[j], o["P"][j]) <= 1e-12, (j, rel(P[j], o["P"][j]))
            for key in ("G", "ctil", "atil"):
                assert rel(g[key], o[key]) <= 1e-10, (k, key, rel(g[key], o[key]))
            x = host(g["x"])
            assert rel(x, o["x"]) <= 1e-10, k


@pytest.mark.parametrize("name", ["rec_s16_ragged", "apply_s16_odd", "rec_s7_odd"])
def test_pairs_fp32_inner_step(hip, name):
    """FP32 basis by pairs: the FP32 Gram matrix of one step within 1e-4 of
    the oracle's FP64 one (the FP32 single-step path meets the same bound),
    and a FP32+IR solve to 1e-8 within 1.5x the FP64 outer iterations."""
    (nx, ny, nz), s, nu, extra = CASES[name]
    pr = gen.small_poisson3d(nx, ny, nz, seed=len(name))
    A, b = oracle_rhs(pr)
    bt = t64(b)
    m = s - 1 if extra.get("gram") == "apply" else s
    x = np.zeros(pr.n)
    with hip.Solver(hip.Operator.stencil(nx, ny, nz), s, nu, pr.lmin, pr.lmax, precision="fp32ir",
                    **extra) as sv:
        assert sv.basis_pairs == m // 2
        for k in range(3):
            o = oracle.step(A, b, x, s, nu, pr.lmin, pr.lmax, **_oracle_kw(extra))
            g = sv.step(bt, t64(x))
            assert rel(g["G"], o["G"]) < 1e-4, (k, rel(g["G"], o["G"]))
            x = o["x"]
        x32, st32 = sv.solve(bt, None, 1e-8)
    ref = oracle.solve(A, b, None, s, nu, pr.lmin, pr.lmax, 1e-8, **_oracle_kw(extra))
    assert st32.status == 0
    assert np.linalg.norm(b - oracle.spmv(A, host(x32))) / np.linalg.norm(b) <= 1e-8
    assert st32.outer_iters <= 1.5 * ref["iters"] + 3


def test_pairs_only_where_they_apply(hip):
    """Single steps for every other operator, with AP stored, and for the
    monomial basis."""
    pr = gen.small_poisson3d(30, 20, 10, seed=3)
    with hip.Solver(hip.Operator.stencil(30, 20, 10), 8, 10, pr.lmin, pr.lmax, gram="stored") as sv:
        assert sv.basis_pairs == 0 and sv.basis_launches == 8
    with hip.Solver(hip.Operator.stencil(30, 20, 10), 8, 10, pr.lmin, pr.lmax, basis="monomial") as sv:
        assert sv.basis_pairs == 0
    with hip.Solver(make_operator(hip, pr, "csr"), 8, 10, pr.lmin, pr.lmax) as sv:
        assert sv.basis_pairs == 0
    pf = gen.small_faces3d(12, 11, 10, seed=4, sigma=0.5)
    with hip.Solver(make_operator(hip, pf, "stencil"), 8, 10, pf.lmin, pf.lmax) as sv:
        assert sv.basis_pairs == 0
    p27 = gen.small_poisson27(12, 11, 10, seed=5)
    with hip.Solver(make_operator(hip, p27, "stencil"), 8, 10, p27.lmin, p27.lmax) as sv:
        assert sv.basis_pairs == 0
