"""Batched solves (many uneven stencil systems x several right-hand sides per
launch) against the FP64 oracle, pair by pair, with both Gram kinds a
batched context takes: the recurrence kind (default for s <= 31: the basis
keeps p_s, the matrix-core kernel forms the M-weighted Gram of p_0 .. p_s
per pair, the FGS kernel maps it onto P^T A P) and the stored-AP kind."""
import numpy as np
import pytest
import torch

import gen
import oracle
from helpers import rel

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def t64(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def host(t):
    return t.detach().cpu().numpy()


def make_batch(seed, dims_list, nrhs, faces=True, sigma=1.0):
    r = gen.rng(seed)
    systems = []
    for dims in dims_list:
        nx, ny, nz = dims
        if faces:
            kx, ky, kz = gen.face_coefficients(r, nx, ny, nz, sigma)
            lmin, lmax = gen.gershgorin_jacobi_bounds()
        else:
            kx = ky = kz = None
            lmin, lmax = gen.jacobi_poisson_bounds(nx, ny, nz)
        systems.append(dict(dims=dims, kx=kx, ky=ky, kz=kz, lmin=lmin, lmax=lmax))
    for sy in systems:
        n = int(np.prod(sy["dims"]))
        sy["rhs"] = np.stack([gen.uniform(r, n) for _ in range(nrhs)])
        sy["A"] = oracle.assemble_stencil7(*sy["dims"], sy["kx"], sy["ky"], sy["kz"])
    return systems


def run_batched(hip, systems, nrhs, s, nu, tol=1e-8, **kw):
    ops = [hip.Operator.stencil(*sy["dims"], sy["kx"], sy["ky"], sy["kz"]) for sy in systems]
    with hip.BatchedSolver(ops, nrhs, s, nu, [sy["lmin"] for sy in systems], [sy["lmax"] for sy in systems],
                           **kw) as bs:
        b = [t64(sy["rhs"].ravel()) for sy in systems]
        x, st = bs.solve(b, None, tol, raise_on_error=False)
    return [host(xq).reshape(nrhs, -1) for xq in x], st


@pytest.mark.parametrize("gram", ["auto", "stored"])
@pytest.mark.parametrize("faces", [True, False])
def test_batched_fp64_matches_oracle_per_pair(hip, faces, gram):
    dims = [(10, 9, 8), (13, 12, 11), (7, 7, 7), (16, 5, 9)]
    nrhs, s, nu = 3, 8, 25
    systems = make_batch(1, dims, nrhs, faces=faces)
    x, st = run_batched(hip, systems, nrhs, s, nu, gram=gram)
    for q, sy in enumerate(systems):
        for r in range(nrhs):
            b = sy["rhs"][r]
            ref = oracle.solve(sy["A"], b, None, s, nu, sy["lmin"], sy["lmax"], 1e-8)
            p = st[q * nrhs + r]
            true_rel = np.linalg.norm(b - oracle.spmv(sy["A"], x[q][r])) / np.linalg.norm(b)
            assert p.status == 0 and true_rel <= 1e-8, (q, r, p.status, true_rel)
            assert abs(p.outer_iters - ref["iters"]) <= max(1, int(0.05 * ref["iters"])), (q, r)


# (s, faces, precond, gram): widths on both sides of the matrix-core column
# blocks (17 and 20 columns with the recurrence kind), Jacobi off
FIRST_ITERATES = {
    "s6_faces_rec": (6, True, True, "auto"),
    "s6_faces_stored": (6, True, True, "stored"),
    "s16_poisson_rec": (16, False, True, "auto"),
    "s19_faces_rec": (19, True, True, "recurrence"),
    "s8_faces_no_jacobi_rec": (8, True, False, "auto"),
    "s8_poisson_no_jacobi_rec": (8, False, False, "auto"),
}


@pytest.mark.parametrize("name", list(FIRST_ITERATES))
def test_batched_first_iterates_follow_oracle(hip, name):
    s, faces, precond, gram = FIRST_ITERATES[name]
    dims = [(11, 10, 9), (6, 8, 7)]
    nrhs, nu = 2, 20
    systems = make_batch(2, dims, nrhs, faces=faces)
    for k in (1, 2, 3):
        x, st = run_batched(hip, systems, nrhs, s, nu, max_outer=k, precond=precond, gram=gram)
        for q, sy in enumerate(systems):
            for r in range(nrhs):
                assert st[q * nrhs + r].outer_iters == k and st[q * nrhs + r].status == 5
                xo = np.zeros(sy["rhs"].shape[1])
                for _ in range(k):
                    xo = oracle.step(sy["A"], sy["rhs"][r], xo, s, nu, sy["lmin"], sy["lmax"],
                                     precond=1 if precond else 0)["x"]
                assert rel(x[q][r], xo) <= 1e-10, (k, q, r)


@pytest.mark.parametrize("gram", ["auto", "stored"])
def test_batched_fp32ir_reaches_tolerance(hip, gram):
    dims = [(12, 12, 12), (9, 14, 10), (20, 6, 6)]
    nrhs, s, nu = 4, 16, 25
    systems = make_batch(3, dims, nrhs)
    x, st = run_batched(hip, systems, nrhs, s, nu, precision="fp32ir", gram=gram)
    for q, sy in enumerate(systems):
        for r in range(nrhs):
            b = sy["rhs"][r]
            assert st[q * nrhs + r].status == 0
            assert np.linalg.norm(b - oracle.spmv(sy["A"], x[q][r])) <= 1e-8 * np.linalg.norm(b)


def test_batched_pairs_converge_independently(hip):
    """A zero right-hand side stops at once; the other pairs of the same
    system are unaffected."""
    dims = [(8, 8, 8), (10, 7, 9)]
    nrhs, s, nu = 3, 8, 25
    systems = make_batch(4, dims, nrhs)
    systems[0]["rhs"][1] = 0.0
    x, st = run_batched(hip, systems, nrhs, s, nu)
    assert st[1].outer_iters == 0 and np.all(x[0][1] == 0)
    for q, sy in enumerate(systems):
        for r in range(nrhs):
            b = sy["rhs"][r]
            if np.linalg.norm(b) > 0:
                assert np.linalg.norm(b - oracle.spmv(sy["A"], x[q][r])) <= 1e-8 * np.linalg.norm(b)


def test_batched_uneven_c4_like(hip):
    """The batched workload's recipe at reduced size: grids N ~ U{12..24},
    log-normal faces (sigma = 1), 8 right-hand sides, s = 16, nu = 25."""
    probs = gen.config4(seed=0, nsys=6, nrhs=8, nmin=12, nmax=24)
    nrhs, s, nu = 8, 16, 25
    ops = [hip.Operator.stencil(*pr.dims, pr.kx, pr.ky, pr.kz) for pr in probs]
    with hip.BatchedSolver(ops, nrhs, s, nu, [pr.lmin for pr in probs], [pr.lmax for pr in probs]) as bs:
        b = [t64(np.concatenate(pr.rhs)) for pr in probs]
        x, st = bs.solve(b, None, 1e-8)
    for q, pr in enumerate(probs):
        A = oracle.problem_csr(pr)
        xq = host(x[q]).reshape(nrhs, -1)
        for r in range(nrhs):
            assert np.linalg.norm(pr.rhs[r] - oracle.spmv(A, xq[r])) <= 1e-8 * np.linalg.norm(pr.rhs[r])


def test_batched_setup_rejects_csr_and_mixed(hip):
    pr = gen.small_faces3d(5, 5, 5)
    rp, ci, v = pr.csr()
    with pytest.raises(hip.SStepError) as ei:
        hip.BatchedSolver([hip.Operator.csr(rp, ci, v)], 1, 4, 5, [0.0], [2.0])
    assert ei.value.name == "SSTEP_E_UNSUPPORTED"
    with pytest.raises(hip.SStepError) as ei:
        hip.BatchedSolver([hip.Operator.stencil(5, 5, 5, pr.kx, pr.ky, pr.kz), hip.Operator.stencil(4, 4, 4)],
                          1, 4, 5, [0.0, 0.0], [2.0, 2.0])
    assert ei.value.name == "SSTEP_E_ARG"


def test_batched_gram_kind_selection(hip):
    pr = gen.small_faces3d(6, 5, 4)
    ops = [hip.Operator.stencil(6, 5, 4, pr.kx, pr.ky, pr.kz)]
    with hip.BatchedSolver(ops, 2, 8, 5, [0.0], [2.0]) as bs:
        assert bs.gram_kind == "moments"
    with hip.BatchedSolver(ops, 2, 8, 5, [0.0], [2.0], gram="recurrence") as bs:
        assert bs.gram_kind == "recurrence"
    with hip.BatchedSolver(ops, 2, 8, 5, [0.0], [2.0], gram="stored") as bs:
        assert bs.gram_kind == "stored"
    with hip.BatchedSolver(ops, 2, 32, 5, [0.0], [2.0]) as bs:
        assert bs.gram_kind == "stored"
    with hip.BatchedSolver(ops, 2, 7, 5, [0.0], [2.0]) as bs:
        assert bs.gram_kind == "recurrence"
    with pytest.raises(hip.SStepError) as ei:
        hip.BatchedSolver(ops, 2, 8, 5, [0.0], [2.0], gram="apply")
    assert ei.value.name == "SSTEP_E_UNSUPPORTED"
    with pytest.raises(hip.SStepError) as ei:
        hip.BatchedSolver(ops, 2, 32, 5, [0.0], [2.0], gram="recurrence")
    assert ei.value.name == "SSTEP_E_UNSUPPORTED"
