"""CSR operators with irregular rows on the GPU against the oracle.

The library keeps a CSR operator also as sliced ELL (slices of 64 rows, each
as wide as its longest row, padding skipped), so row lengths that differ
strongly inside a slice and a partial last slice are the cases that matter.  The matrix is a seeded random symmetric one,
strictly diagonally dominant with a positive diagonal (so SPD), row lengths
from 6 to 62; the Jacobi-preconditioned spectrum lies in (0, 2), the
bounds used.  Checked through the C ABI: the product entry by entry, lockstep
outer iterations (1e-10), solves to 1e-8 in FP64 and FP32+IR, and the same
after new coefficients on the same pattern."""
import numpy as np
import pytest
import torch

import oracle
from helpers import rel

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def t64(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def host(t):
    return t.detach().cpu().numpy()


def random_spd_csr(n, seed, max_off=30):
    """Symmetric pattern: row i draws k_i ~ U{0..max_off} partners; the union
    with its transpose is taken, values ~ U[-1, 1] mirrored, diagonal
    1 + sum of |off-diagonal| of the row."""
    r = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        k = int(r.integers(0, max_off + 1))
        js = r.choice(n, size=k, replace=False)
        js = js[js != i]
        rows.extend([i] * len(js))
        cols.extend(js.tolist())
    rows, cols = np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64)
    # symmetric pattern, one value per unordered pair
    lo, hi = np.minimum(rows, cols), np.maximum(rows, cols)
    pairs = np.unique(lo * n + hi)
    lo, hi = pairs // n, pairs % n
    v = r.uniform(-1.0, 1.0, size=pairs.size)
    R = np.concatenate([lo, hi])
    C = np.concatenate([hi, lo])
    V = np.concatenate([v, v])
    diag = np.ones(n)
    np.add.at(diag, R, np.abs(V))
    R = np.concatenate([R, np.arange(n)])
    C = np.concatenate([C, np.arange(n)])
    V = np.concatenate([V, diag])
    order = np.lexsort((C, R))
    R, C, V = R[order], C[order], V[order]
    rp = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rp, R + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    return rp, C.astype(np.int32), V


@pytest.fixture(scope="module")
def mat():
    n = 5000  # 78 full slices of 64 rows and a partial one
    rp, ci, v = random_spd_csr(n, seed=31)
    lens = np.diff(rp)
    assert lens.max() >= 40 and lens.max() > 4 * lens.min()  # strongly irregular
    return n, rp, ci, v


def test_apply_entry_by_entry(hip, mat):
    n, rp, ci, v = mat
    x = np.random.default_rng(1).uniform(-1, 1, n)
    A = (rp, ci, v)
    y_ref = oracle.spmv(A, x)
    scale = np.zeros(n)
    np.add.at(scale, np.repeat(np.arange(n), np.diff(rp)), np.abs(v) * np.abs(x[ci]))
    with hip.Solver(hip.Operator.csr(rp, ci, v), 8, 10, 0.0, 2.0) as sv:
        y = host(sv.apply(t64(x)))
    assert np.all(np.abs(y - y_ref) <= 1e-14 * scale + 1e-300)


@pytest.mark.parametrize("s", [5, 8])
def test_lockstep_and_solve(hip, mat, s):
    n, rp, ci, v = mat
    A = (rp, ci, v)
    xs = np.random.default_rng(2).uniform(-1, 1, n)
    b = oracle.spmv(A, xs)
    bt = t64(b)
    x = np.zeros(n)
    with hip.Solver(hip.Operator.csr(rp, ci, v), s, 20, 0.0, 2.0) as sv:
        for k in range(3):
            g = sv.step(bt, t64(x), want_basis=(k == 0))
            o = oracle.step(A, b, x, s, 20, 0.0, 2.0, want_basis=(k == 0))
            assert o["status"] == 0
            if k == 0:
                P = host(g["P"])
                for j in range(s):
                    assert rel(P[j], o["P"][j]) <= 1e-12, j
            for key in ("G", "ctil", "atil"):
                assert rel(g[key], o[key]) <= 1e-10, (k, key, rel(g[key], o[key]))
            x = host(g["x"])
            assert rel(x, o["x"]) <= 1e-10, k
        xg, st = sv.solve(bt, None, 1e-8)
    ref = oracle.solve(A, b, None, s, 20, 0.0, 2.0, 1e-8)
    assert st.status == 0 and ref["status"] == 0
    assert np.linalg.norm(b - oracle.spmv(A, host(xg))) / np.linalg.norm(b) <= 1e-8
    assert abs(st.outer_iters - ref["iters"]) <= max(1, int(0.05 * ref["iters"])), (st.outer_iters, ref["iters"])


def test_fp32ir_and_new_coefficients(hip, mat):
    n, rp, ci, v = mat
    A = (rp, ci, v)
    xs = np.random.default_rng(3).uniform(-1, 1, n)
    b = oracle.spmv(A, xs)
    # new values on the same pattern: the off-diagonal entries scaled by 0.5
    # and the diagonal kept, still strictly diagonally dominant
    is_diag = ci == np.repeat(np.arange(n), np.diff(rp))
    v2 = np.where(is_diag, v, 0.5 * v)
    A2 = (rp, ci, v2)
    b2 = oracle.spmv(A2, xs)
    with hip.Solver(hip.Operator.csr(rp, ci, v), 8, 20, 0.0, 2.0, precision="fp32ir") as sv:
        x, st = sv.solve(t64(b), None, 1e-8)
        assert st.status == 0
        assert np.linalg.norm(b - oracle.spmv(A, host(x))) / np.linalg.norm(b) <= 1e-8
        sv.update_coefficients(hip.Operator.csr(rp, ci, v2))
        y = host(sv.apply(t64(xs)))
        assert rel(y, b2) <= 1e-14
        x2, st2 = sv.solve(t64(b2), None, 1e-8)
        assert st2.status == 0
        assert np.linalg.norm(b2 - oracle.spmv(A2, host(x2))) / np.linalg.norm(b2) <= 1e-8
