"""Two basis steps per launch in batched solves, on the GPU, with the
recurrence Gram kind and with the moments kind (the FP64 default for even s,
whose products the two-step kernel sums per band).

A block of the two-step kernel owns a band of whole grid rows of one system
and a range of its planes; it also forms the first step on the row below and
the row above the band.  The grids here span:
- planes that fit one block (one band);
- several bands, with heights that do not divide the grid;
- rows of 341 points, the widest that still leave one band row per block;
- several z-ranges, the last one shorter.
Widths cover even s, odd s (the last column then takes a single step), s = 2
(the first pair only) and s = 1 (no pair).

Each case is checked two ways with the recurrence kind.  First, the iterates
after 1 and 2 outer iterations equal those of the same context built with one
step per launch, bit for bit: both kernels form every value with the same
operations in the same order, and the rest of the iteration is the same
code.  Second, they are checked against the FP64 oracle within the lockstep
bar of 1e-10.  The even-s cases are checked against the oracle with the
moments kind too."""
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


def make_batch(seed, dims_list, nrhs, faces=True):
    r = gen.rng(seed)
    systems = []
    for dims in dims_list:
        if faces:
            kx, ky, kz = gen.face_coefficients(r, *dims, 1.0)
            lmin, lmax = gen.gershgorin_jacobi_bounds()
        else:
            kx = ky = kz = None
            lmin, lmax = gen.jacobi_poisson_bounds(*dims)
        n = int(np.prod(dims))
        rhs = np.stack([gen.uniform(r, n) for _ in range(nrhs)])
        systems.append(dict(dims=dims, kx=kx, ky=ky, kz=kz, lmin=lmin, lmax=lmax, rhs=rhs))
    return systems


def iterate(hip, systems, nrhs, s, nu, k, **kw):
    """x after k outer iterations of every pair, and the context's basis
    launch counts."""
    ops = [hip.Operator.stencil(*sy["dims"], sy["kx"], sy["ky"], sy["kz"]) for sy in systems]
    with hip.BatchedSolver(ops, nrhs, s, nu, [sy["lmin"] for sy in systems], [sy["lmax"] for sy in systems],
                           max_outer=k, autotune=False, **kw) as bs:
        b = [t64(sy["rhs"].ravel()) for sy in systems]
        x, st = bs.solve(b, None, 1e-14, raise_on_error=False)
        counts = (bs.basis_launches, bs.basis_pairs)
    for p in st:
        assert p.outer_iters == k and p.status == 5, (p.outer_iters, p.status)
    return [host(xq).reshape(nrhs, -1) for xq in x], counts


# name: (grids, nrhs, s, faces, precond)
CASES = {
    # 40 x 37 planes: bands of 19 rows (2 bands), 35 planes: ranges 12, 12, 11
    "faces_bands_ranges_s16": ([(40, 37, 35), (9, 11, 7)], 3, 16, True, True),
    # rows of 341 points: one band row per block, 7 bands
    "faces_widest_rows_s6": ([(341, 7, 5), (20, 20, 20)], 2, 6, True, True),
    # odd s: seven pairs and a single step; heights 63 / 2 bands of 32
    "faces_odd_s15": ([(30, 63, 17), (17, 3, 40)], 2, 15, True, True),
    "poisson_bands_s8": ([(64, 45, 33), (33, 31, 9)], 2, 8, False, True),
    "faces_no_jacobi_s10": ([(50, 29, 18)], 3, 10, True, False),
    "faces_s2_first_pair_only": ([(45, 40, 21)], 2, 2, True, True),
    "faces_s3_pair_and_step": ([(26, 41, 19)], 2, 3, True, True),
}


@pytest.mark.parametrize("name", list(CASES))
def test_pairs_equal_single_steps_and_oracle(hip, name):
    dims, nrhs, s, faces, precond = CASES[name]
    nu = 20
    systems = make_batch(7, dims, nrhs, faces=faces)
    for k in (1, 2):
        # the same Gram kind on both sides (one step per launch has no moments kind)
        x2, c2 = iterate(hip, systems, nrhs, s, nu, k, precond=precond, gram="recurrence")
        x1, c1 = iterate(hip, systems, nrhs, s, nu, k, precond=precond, basis_steps=1, gram="recurrence")
        assert c2 == (s - s // 2, s // 2), c2
        assert c1 == (s, 0), c1
        for q in range(len(systems)):
            assert np.array_equal(x2[q], x1[q]), (k, q, float(np.max(np.abs(x2[q] - x1[q]))))
    # lockstep against the oracle after 2 outer iterations
    for q, sy in enumerate(systems):
        A = oracle.assemble_stencil7(*sy["dims"], sy["kx"], sy["ky"], sy["kz"])
        for r in range(nrhs):
            xo = np.zeros(sy["rhs"].shape[1])
            for _ in range(2):
                o = oracle.step(A, sy["rhs"][r], xo, s, nu, sy["lmin"], sy["lmax"], precond=1 if precond else 0)
                xo = o["x"]
            assert rel(x2[q][r], xo) <= 1e-10, (q, r, rel(x2[q][r], xo))


@pytest.mark.parametrize("name", [k for k, v in CASES.items() if v[2] % 2 == 0])
def test_moments_kind_lockstep(hip, name):
    """The moments kind (FP64 default for even s): the two-step basis sums
    each pair's products per band, the FGS kernel forms the Gram matrix from
    the Chebyshev moments.  x after 1 and 2 outer iterations within 1e-10 of
    the oracle's, pair by pair."""
    dims, nrhs, s, faces, precond = CASES[name]
    nu = 20
    systems = make_batch(7, dims, nrhs, faces=faces)
    ops = [hip.Operator.stencil(*sy["dims"], sy["kx"], sy["ky"], sy["kz"]) for sy in systems]
    with hip.BatchedSolver(ops, nrhs, s, nu, [sy["lmin"] for sy in systems], [sy["lmax"] for sy in systems],
                           autotune=False, precond=precond) as bs:
        assert bs.gram_kind == "moments"
    for k in (1, 2):
        x, _ = iterate(hip, systems, nrhs, s, nu, k, precond=precond)
        for q, sy in enumerate(systems):
            A = oracle.assemble_stencil7(*sy["dims"], sy["kx"], sy["ky"], sy["kz"])
            for r in range(nrhs):
                xo = np.zeros(sy["rhs"].shape[1])
                for _ in range(k):
                    xo = oracle.step(A, sy["rhs"][r], xo, s, nu, sy["lmin"], sy["lmax"],
                                     precond=1 if precond else 0)["x"]
                assert rel(x[q][r], xo) <= 1e-10, (k, q, r, rel(x[q][r], xo))


def test_moments_kind_solve_and_selection(hip):
    """A batched moments solve reaches 1e-8 on every pair; AUTO takes the
    recurrence kind for odd s, FP32+IR and single steps, and the moments
    kind is refused there."""
    systems = make_batch(11, [(40, 37, 35), (21, 19, 17), (12, 12, 12)], 2)
    ops = [hip.Operator.stencil(*sy["dims"], sy["kx"], sy["ky"], sy["kz"]) for sy in systems]
    lo, hi = [sy["lmin"] for sy in systems], [sy["lmax"] for sy in systems]
    with hip.BatchedSolver(ops, 2, 16, 25, lo, hi, autotune=False) as bs:
        assert bs.gram_kind == "moments"
        x, st = bs.solve([t64(sy["rhs"].ravel()) for sy in systems], None, 1e-8)
    for q, sy in enumerate(systems):
        A = oracle.assemble_stencil7(*sy["dims"], sy["kx"], sy["ky"], sy["kz"])
        xq = host(x[q]).reshape(2, -1)
        for r in range(2):
            b = sy["rhs"][r]
            assert st[q * 2 + r].status == 0
            assert np.linalg.norm(b - oracle.spmv(A, xq[r])) <= 1e-8 * np.linalg.norm(b)
    for kw in ({"s": 15}, {"precision": "fp32ir"}, {"basis_steps": 1}):
        s = kw.pop("s", 16)
        with hip.BatchedSolver(ops, 2, s, 25, lo, hi, autotune=False, **kw) as bs:
            assert bs.gram_kind == "recurrence", kw
        with pytest.raises(hip.SStepError) as e:
            hip.BatchedSolver(ops, 2, s, 25, lo, hi, autotune=False, gram="moments", **kw)
        assert e.value.name == "SSTEP_E_UNSUPPORTED"


def test_whole_system_ranges(hip):
    """A batch big enough for 4 blocks per CU: 64 systems of side 36..48
    with 8 right-hand sides, so each system is one z-range of up to 48
    planes (the smaller batches above take ranges of about 16).  The first
    iterate of four pairs against the oracle's to 1e-10, and every pair's
    solve to 1e-8.  Once pairs stop, fewer than 4 blocks per CU are left and
    the solve moves to ranges of 16 planes: with the recurrence Gram kind
    (whose sums do not depend on the bands) that solve equals one basis step
    per launch bit for bit, and an FP32+IR solve that moves too reaches 1e-8
    in every pair."""
    probs = gen.config4(seed=3, nsys=64, nrhs=8, nmin=36, nmax=48)
    nrhs, s, nu = 8, 16, 25
    ops = [hip.Operator.stencil(*pr.dims, pr.kx, pr.ky, pr.kz) for pr in probs]
    lo, hi = [pr.lmin for pr in probs], [pr.lmax for pr in probs]
    b = [t64(np.concatenate(pr.rhs)) for pr in probs]
    with hip.BatchedSolver(ops, nrhs, s, nu, lo, hi, autotune=False, max_outer=1) as bs:
        assert bs.basis_pairs == 8 and bs.gram_kind == "moments"
        x1, _ = bs.solve(b, None, 1e-14, raise_on_error=False)
    for q, r in ((0, 0), (17, 3), (40, 7), (63, 5)):
        pr = probs[q]
        A = oracle.problem_csr(pr)
        xo = oracle.step(A, pr.rhs[r], np.zeros(pr.n), s, nu, pr.lmin, pr.lmax)["x"]
        assert rel(host(x1[q]).reshape(nrhs, -1)[r], xo) <= 1e-10, (q, r)
    with hip.BatchedSolver(ops, nrhs, s, nu, lo, hi, autotune=False) as bs:
        x, st = bs.solve(b, None, 1e-8)
        bands, tail, replays = bs.bands()
    assert tail > bands >= 64 and replays > 0, (bands, tail, replays)
    for q, pr in enumerate(probs):
        A = oracle.problem_csr(pr)
        xq = host(x[q]).reshape(nrhs, -1)
        for r in range(nrhs):
            assert st[q * nrhs + r].status == 0
            assert np.linalg.norm(pr.rhs[r] - oracle.spmv(A, xq[r])) <= 1e-8 * np.linalg.norm(pr.rhs[r]), (q, r)
    runs = []
    for steps in (0, 1):
        with hip.BatchedSolver(ops, nrhs, s, nu, lo, hi, autotune=False, gram="recurrence", basis_steps=steps) as bs:
            xr, sr = bs.solve(b, None, 1e-8)
            runs.append(([host(v) for v in xr], [t.outer_iters for t in sr], bs.bands()))
    assert runs[0][2][2] > 0 and runs[1][2] == (0, 0, 0), (runs[0][2], runs[1][2])
    assert runs[0][1] == runs[1][1]
    for q in range(len(probs)):
        assert np.array_equal(runs[0][0][q], runs[1][0][q]), q
    # FP32 basis (recurrence kind) on both tables: every pair to 1e-8 in the FP64 residual
    ops32 = [hip.Operator.stencil(*pr.dims, pr.kx, pr.ky, pr.kz) for pr in probs]
    with hip.BatchedSolver(ops32, nrhs, s, nu, lo, hi, autotune=False, precision="fp32ir") as bs:
        x, st = bs.solve(b, None, 1e-8)
        assert bs.gram_kind == "recurrence" and bs.bands()[2] > 0, bs.bands()
    for q, pr in enumerate(probs):
        A = oracle.problem_csr(pr)
        xq = host(x[q]).reshape(nrhs, -1)
        for r in range(nrhs):
            assert st[q * nrhs + r].status == 0
            assert np.linalg.norm(pr.rhs[r] - oracle.spmv(A, xq[r])) <= 1e-8 * np.linalg.norm(pr.rhs[r]), (q, r)


def test_pairs_fp32ir_solve(hip):
    """FP32 basis by pairs (FP32 face coefficients): every pair reaches 1e-8
    in the FP64 residual."""
    dims = [(40, 37, 35), (33, 20, 18), (12, 12, 12)]
    nrhs, s, nu = 2, 16, 25
    systems = make_batch(8, dims, nrhs)
    ops = [hip.Operator.stencil(*sy["dims"], sy["kx"], sy["ky"], sy["kz"]) for sy in systems]
    with hip.BatchedSolver(ops, nrhs, s, nu, [0.0] * 3, [2.0] * 3, precision="fp32ir", autotune=False) as bs:
        assert bs.basis_pairs == 8
        x, st = bs.solve([t64(sy["rhs"].ravel()) for sy in systems], None, 1e-8)
    for q, sy in enumerate(systems):
        A = oracle.assemble_stencil7(*sy["dims"], sy["kx"], sy["ky"], sy["kz"])
        xq = host(x[q]).reshape(nrhs, -1)
        for r in range(nrhs):
            assert st[q * nrhs + r].status == 0
            b = sy["rhs"][r]
            assert np.linalg.norm(b - oracle.spmv(A, xq[r])) <= 1e-8 * np.linalg.norm(b)


def test_pairs_only_where_they_fit(hip):
    """One step per launch with AP stored, and for a batch holding a system
    whose rows are too wide for a band (342 points); s = 1 has no pair."""
    small = make_batch(9, [(12, 10, 8)], 1)[0]
    wide = make_batch(9, [(342, 3, 3)], 1)[0]

    def counts(systems, s, **kw):
        ops = [hip.Operator.stencil(*sy["dims"], sy["kx"], sy["ky"], sy["kz"]) for sy in systems]
        with hip.BatchedSolver(ops, 1, s, 5, [0.0] * len(ops), [2.0] * len(ops), autotune=False, **kw) as bs:
            return bs.basis_launches, bs.basis_pairs

    assert counts([small], 8) == (4, 4)
    assert counts([small], 8, gram="stored") == (8, 0)
    assert counts([small, wide], 8) == (8, 0)
    assert counts([small], 1) == (1, 0)
    with pytest.raises(hip.SStepError) as ei:
        counts([small], 8, basis_steps=2)
    assert ei.value.name == "SSTEP_E_ARG"


def test_autotuned_tile_schedule(hip, tmp_path, monkeypatch):
    """A batch of 1.1M unknowns is autotuned at set-up: the tuner times the
    residual and the update on scratch iterates, then gives the pairs back.
    The schedule is one of its candidates, the cache holds it under the
    iteration-timed key, and every pair still reaches 1e-8 (checked against
    the oracle's operator); a second set-up reads the same schedule back."""
    monkeypatch.setenv("SSTEP_TUNE_CACHE", str(tmp_path / "tune.json"))
    probs = gen.config4(seed=5, nsys=8, nrhs=2, nmin=50, nmax=54)
    assert sum(pr.n for pr in probs) >= 1 << 20
    nrhs, s, nu = 2, 16, 25
    ops = [hip.Operator.stencil(*pr.dims, pr.kx, pr.ky, pr.kz) for pr in probs]
    lo, hi = [pr.lmin for pr in probs], [pr.lmax for pr in probs]
    b = [t64(np.concatenate(pr.rhs[:nrhs])) for pr in probs]
    with hip.BatchedSolver(ops, nrhs, s, nu, lo, hi) as bs:
        tiles = dict(bs.tiles)
        x, st = bs.solve(b, None, 1e-8)
    assert tiles["rows_per_tile"] in (2048, 8192, 32768) and tiles["grid_factor"] in (2, 4, 8), tiles
    text = (tmp_path / "tune.json").read_text()
    assert "timed=iteration" in text and "batched" in text
    for q, pr in enumerate(probs):
        A = oracle.problem_csr(pr)
        xq = host(x[q]).reshape(nrhs, -1)
        for r in range(nrhs):
            assert st[q * nrhs + r].status == 0
            assert np.linalg.norm(pr.rhs[r] - oracle.spmv(A, xq[r])) <= 1e-8 * np.linalg.norm(pr.rhs[r]), (q, r)
    with hip.BatchedSolver(ops, nrhs, s, nu, lo, hi) as bs:
        assert dict(bs.tiles) == tiles


def test_constant_poisson_batch_moments(hip):
    """Constant-coefficient 7-point systems (no face arrays) on the default
    kind: the moments kind with two steps per launch and the band-table
    residual.  One band (a 12 x 10 plane), several bands (40 x 30) and a
    narrow grid (36 x 7).  The first iterate of every pair against the
    oracle's to 1e-10, and every pair's solve to 1e-8."""
    dims = [(12, 10, 9), (40, 30, 20), (36, 7, 33)]
    nrhs, s, nu = 2, 16, 25
    probs = [gen.small_poisson3d(*d, seed=7 + q) for q, d in enumerate(dims)]
    ops = [hip.Operator.stencil(*d) for d in dims]
    lo, hi = [pr.lmin for pr in probs], [pr.lmax for pr in probs]
    rng = np.random.default_rng(11)
    rhs = [[rng.uniform(-1.0, 1.0, pr.n) for _ in range(nrhs)] for pr in probs]
    b = [t64(np.concatenate(rq)) for rq in rhs]
    with hip.BatchedSolver(ops, nrhs, s, nu, lo, hi, autotune=False, max_outer=1) as bs:
        assert bs.gram_kind == "moments" and bs.basis_pairs == s // 2
        x1, _ = bs.solve(b, None, 1e-14, raise_on_error=False)
    for q, pr in enumerate(probs):
        A = oracle.problem_csr(pr)
        for r in range(nrhs):
            xo = oracle.step(A, rhs[q][r], np.zeros(pr.n), s, nu, pr.lmin, pr.lmax)["x"]
            assert rel(host(x1[q]).reshape(nrhs, -1)[r], xo) <= 1e-10, (q, r)
    with hip.BatchedSolver(ops, nrhs, s, nu, lo, hi, autotune=False) as bs:
        x, st = bs.solve(b, None, 1e-8)
    for q, pr in enumerate(probs):
        A = oracle.problem_csr(pr)
        xq = host(x[q]).reshape(nrhs, -1)
        for r in range(nrhs):
            assert st[q * nrhs + r].status == 0
            assert np.linalg.norm(rhs[q][r] - oracle.spmv(A, xq[r])) <= 1e-8 * np.linalg.norm(rhs[q][r]), (q, r)
