"""The Gram kernel that forms A p_j itself (stencil operators, s <= 16, AP not
kept) against the stored-AP Gram kernel and the FP64 oracle, through the C ABI.

Both kernels compute the same sums in different orders, so per outer
iteration they agree to rounding: G, ctil, atil and x_{k+1} within 1e-12
relative of each other, and each within 1e-10 of the oracle.
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


PROBLEMS = {
    "poisson_ragged": lambda: ragged_poisson(0),
    "faces_23x17x13": lambda: gen.small_faces3d(23, 17, 13, seed=2, sigma=1.0),
    "faces_5x40x3": lambda: gen.small_faces3d(5, 40, 3, seed=6, sigma=0.5),
}


def test_gram_mode_selection(hip):
    """The default is the moments kind for s <= 31 in FP64 (every operator,
    p_0 = M^{-1} r), the recurrence kind in FP32+IR, the stored-AP kind at
    s = 32; the other kinds on request."""
    pr = ragged_poisson(0)
    op = make_operator(hip, pr, "stencil")
    with hip.Solver(op, 16, 5, pr.lmin, pr.lmax) as sv:
        assert sv.gram_kind == "moments" and not sv.gram_applies_operator
    with hip.Solver(op, 16, 5, pr.lmin, pr.lmax, gram="recurrence") as sv:
        assert sv.gram_kind == "recurrence" and not sv.gram_applies_operator
    with hip.Solver(op, 16, 5, pr.lmin, pr.lmax, gram="apply") as sv:
        assert sv.gram_kind == "apply" and sv.gram_applies_operator
    with hip.Solver(op, 16, 5, pr.lmin, pr.lmax, gram="stored") as sv:
        assert sv.gram_kind == "stored"
    with hip.Solver(op, 16, 5, pr.lmin, pr.lmax, precision="fp32ir") as sv:
        assert sv.gram_kind == "recurrence"
    with hip.Solver(op, 16, 5, pr.lmin, pr.lmax, precision="fp32ir", gram="apply") as sv:
        assert sv.gram_kind == "apply"
    with hip.Solver(op, 17, 5, pr.lmin, pr.lmax) as sv:
        assert sv.gram_kind == "moments"
    with hip.Solver(op, 32, 5, pr.lmin, pr.lmax) as sv:
        assert sv.gram_kind == "stored"
    with hip.Solver(make_operator(hip, pr, "csr"), 8, 5, pr.lmin, pr.lmax) as sv:
        assert sv.gram_kind == "moments"


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("s", [1, 4, 8, 9, 13, 16])
def test_lockstep_matches_stored_ap_and_oracle(hip, name, s):
    pr = PROBLEMS[name]()
    nu = 20
    A, b = oracle_rhs(pr)
    bt = t64(b)
    x = np.zeros(pr.n)
    op = make_operator(hip, pr, "stencil")
    with hip.Solver(op, s, nu, pr.lmin, pr.lmax, gram="apply") as fused, \
            hip.Solver(op, s, nu, pr.lmin, pr.lmax, gram="stored") as stored, \
            hip.Solver(op, s, nu, pr.lmin, pr.lmax, gram="recurrence") as recur:
        assert fused.gram_applies_operator and not stored.gram_applies_operator
        for k in range(3):
            gf = fused.step(bt, t64(x), want_basis=(k == 0))
            gs = stored.step(bt, t64(x), want_basis=(k == 0))
            gr = recur.step(bt, t64(x))
            o = oracle.step(A, b, x, s, nu, pr.lmin, pr.lmax, want_basis=(k == 0))
            assert o["status"] == 0
            for key in ("G", "ctil", "atil"):
                assert rel(gf[key], gs[key]) <= 1e-12, (k, key, rel(gf[key], gs[key]))
                assert rel(gr[key], gs[key]) <= 1e-12, (k, key, rel(gr[key], gs[key]))
                assert rel(gf[key], o[key]) <= 1e-10, (k, key, rel(gf[key], o[key]))
            xf = host(gf["x"])
            assert rel(xf, host(gs["x"])) <= 1e-12, k
            assert rel(xf, o["x"]) <= 1e-10, k
            if k == 0:
                # the on-demand products of the step entry point equal the stored ones
                assert torch.equal(gf["P"], gs["P"])
                for j in range(s):
                    assert rel(host(gf["AP"])[j], o["AP"][j]) <= 1e-12, j
            x = xf


def test_grid_strided_blocks_match_oracle(hip):
    """A plane of more tiles than blocks: each block loops over several
    (tile, z-range) items."""
    pr = gen.small_poisson3d(512, 520, 2, seed=7)
    s, nu = 16, 25
    A, b = oracle_rhs(pr)
    with hip.Solver(make_operator(hip, pr, "stencil"), s, nu, pr.lmin, pr.lmax, autotune=False, gram="apply") as sv:
        assert sv.gram_applies_operator
        g = sv.step(t64(b), t64(np.zeros(pr.n)))
    o = oracle.step(A, b, np.zeros(pr.n), s, nu, pr.lmin, pr.lmax)
    for key in ("G", "ctil", "atil"):
        assert rel(g[key], o[key]) <= 1e-10, key
    assert rel(host(g["x"]), o["x"]) <= 1e-10


@pytest.mark.parametrize("faces", [False, True])
def test_ragged_tiles_with_multiplane_ranges(hip, faces):
    """Partial tiles in x and y (203 = 6 x 32 + 11, 101 = 12 x 8 + 5) with
    z-ranges of several planes: points outside the grid stay zero while the
    block marches through the range."""
    pr = gen.small_faces3d(203, 101, 60, seed=8, sigma=0.5) if faces else gen.small_poisson3d(203, 101, 60, seed=8)
    s, nu = 16, 25
    A, b = oracle_rhs(pr)
    x = np.zeros(pr.n)
    with hip.Solver(make_operator(hip, pr, "stencil"), s, nu, pr.lmin, pr.lmax, autotune=False, gram="apply") as sv:
        assert sv.gram_applies_operator
        for k in range(2):
            g = sv.step(t64(b), t64(x))
            o = oracle.step(A, b, x, s, nu, pr.lmin, pr.lmax)
            for key in ("G", "ctil", "atil"):
                assert rel(g[key], o[key]) <= 1e-10, (k, key, rel(g[key], o[key]))
            x = host(g["x"])
            assert rel(x, o["x"]) <= 1e-10, k


@pytest.mark.parametrize("gram", ["apply", "stored"])
@pytest.mark.parametrize("precision", ["fp64", "fp32ir"])
@pytest.mark.parametrize("name", ["poisson_ragged", "faces_23x17x13"])
def test_solves_reach_tolerance_in_both_modes(hip, gram, precision, name):
    pr = PROBLEMS[name]()
    A, b = oracle_rhs(pr)
    ref = oracle.solve(A, b, None, 16, 25, pr.lmin, pr.lmax, 1e-8)
    with hip.Solver(make_operator(hip, pr, "stencil"), 16, 25, pr.lmin, pr.lmax, precision=precision,
                    gram=gram) as sv:
        x, st = sv.solve(t64(b), None, 1e-8)
    true_rel = np.linalg.norm(b - oracle.spmv(A, host(x))) / np.linalg.norm(b)
    assert st.status == 0 and true_rel <= 1e-8
    if precision == "fp64":
        assert abs(st.outer_iters - ref["iters"]) <= max(1, int(0.05 * ref["iters"]))


def test_fused_solve_is_bitwise_reproducible(hip):
    pr = gen.small_faces3d(23, 17, 13, seed=2, sigma=1.0)
    A, b = oracle_rhs(pr)
    with hip.Solver(make_operator(hip, pr, "stencil"), 12, 20, pr.lmin, pr.lmax) as sv:
        x1, s1 = sv.solve(t64(b))
        x2, s2 = sv.solve(t64(b))
    assert s1.outer_iters == s2.outer_iters and torch.equal(x1, x2)
