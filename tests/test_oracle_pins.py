"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties one oracle function to something other than itself: closed-form
eigenpairs, the closed form of Chebyshev polynomials, the paper's theorems
(FGS residual structure, backward stability, MGS equivalence), invariants
(energy identity, Galerkin orthogonality, symmetry/definiteness), textbook
special cases (s = 1 steepest descent, Cholesky) and dense direct solves on
tiny grids.  Dense NumPy linear algebra is used only as an independent check.
"""
import math

import numpy as np
import pytest

import gen
import oracle

EPS = np.finfo(np.float64).eps


def dense(A):
    rp, ci, v = A
    n = rp.size - 1
    M = np.zeros((n, n))
    for i in range(n):
        M[i, ci[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    return M


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ---------------------------------------------------------------------------
# P1 / P12: operator assembly and spectral bounds (sine eigenpairs, closed form)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nx,ny", [(7, 5), (64, 64)])
def test_poisson2d_sine_eigenpairs(nx, ny):
    A = gen.poisson2d_csr(nx, ny)
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    for a, b in [(1, 1), (2, 3), (nx, ny), (3, 1)]:
        v = (np.sin(a * math.pi * (i + 1) / (nx + 1)) * np.sin(b * math.pi * (j + 1) / (ny + 1))).ravel()
        lam = 4 - 2 * math.cos(a * math.pi / (nx + 1)) - 2 * math.cos(b * math.pi / (ny + 1))
        # backward-error scale: ||A|| <= 8
        assert np.linalg.norm(oracle.spmv(A, v) - lam * v) < 8 * 1e-14 * np.linalg.norm(v)


@pytest.mark.parametrize("dims", [(5, 4, 3), (9, 9, 9)])
def test_poisson3d_sine_eigenpairs(dims):
    nx, ny, nz = dims
    Ao = oracle.assemble_stencil7(nx, ny, nz)
    Ag = gen.poisson3d_csr(nx, ny, nz)
    # P12-style: the generator's CSR and the oracle's assembly are the same matrix
    for a, b in zip(Ao, Ag):
        assert np.array_equal(a, b)
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    k = np.arange(nz)[:, None, None]
    for a, b, c in [(1, 1, 1), (2, 1, 3), (nx, ny, nz)]:
        v = (np.sin(a * math.pi * (i + 1) / (nx + 1)) * np.sin(b * math.pi * (j + 1) / (ny + 1))
             * np.sin(c * math.pi * (k + 1) / (nz + 1))).ravel()
        lam = 6 - 2 * (math.cos(a * math.pi / (nx + 1)) + math.cos(b * math.pi / (ny + 1))
                       + math.cos(c * math.pi / (nz + 1)))
        assert np.linalg.norm(oracle.spmv(Ao, v) - lam * v) < 12 * 1e-14 * np.linalg.norm(v)


def test_unit_faces_reproduce_poisson_bitwise():
    nx, ny, nz = 6, 5, 4
    ones = [np.ones(nz * ny * (nx + 1)), np.ones(nz * (ny + 1) * nx), np.ones((nz + 1) * ny * nx)]
    A1 = oracle.assemble_stencil7(nx, ny, nz, *ones)
    A0 = oracle.assemble_stencil7(nx, ny, nz)
    for a, b in zip(A1, A0):
        assert np.array_equal(a, b)
    assert oracle.csr_valid(nx * ny * nz, A0)


def test_face_operator_quadratic_form_and_generator():
    """u^T A u equals the sum over faces of k_f (u_p - u_q)^2 (u_q = 0 across the
    boundary), the defining energy of the face operator; the generator's CSR is
    the same matrix."""
    nx, ny, nz = 5, 4, 3
    r = gen.rng(3)
    kx, ky, kz = gen.face_coefficients(r, nx, ny, nz, 1.0)
    A = oracle.assemble_stencil7(nx, ny, nz, kx, ky, kz)
    for a, b in zip(A, gen.faces3d_csr(nx, ny, nz, kx, ky, kz)):
        assert np.array_equal(a, b)
    Ad = dense(A)
    assert np.array_equal(Ad, Ad.T)
    u = r.standard_normal(nx * ny * nz)
    U = np.pad(u.reshape(nz, ny, nx), 1)
    KX = kx.reshape(nz, ny, nx + 1)
    KY = ky.reshape(nz, ny + 1, nx)
    KZ = kz.reshape(nz + 1, ny, nx)
    e = (KX * np.diff(U[1:-1, 1:-1, :], axis=2) ** 2).sum()
    e += (KY * np.diff(U[1:-1, :, 1:-1], axis=1) ** 2).sum()
    e += (KZ * np.diff(U[:, 1:-1, 1:-1], axis=0) ** 2).sum()
    assert abs(u @ Ad @ u - e) < 1e-12 * e


@pytest.mark.parametrize("dims", [(7, 5), (6, 6), (4, 5, 3), (5, 5, 5)])
def test_jacobi_bounds_closed_form(dims):
    A = gen.poisson2d_csr(*dims) if len(dims) == 2 else gen.poisson3d_csr(*dims)
    Ad = dense(A)
    ev = np.linalg.eigvalsh(Ad / np.diag(Ad)[0])
    lmin, lmax = gen.jacobi_poisson_bounds(*dims)
    assert abs(ev[0] - lmin) < 1e-13 and abs(ev[-1] - lmax) < 1e-13


def test_gershgorin_bounds_contain_face_spectrum():
    nx, ny, nz = 5, 4, 3
    kx, ky, kz = gen.face_coefficients(gen.rng(1), nx, ny, nz, 1.0)
    Ad = dense(oracle.assemble_stencil7(nx, ny, nz, kx, ky, kz))
    dh = 1 / np.sqrt(np.diag(Ad))
    ev = np.linalg.eigvalsh(dh[:, None] * Ad * dh[None, :])
    lo, hi = gen.gershgorin_jacobi_bounds()
    assert lo <= ev[0] and ev[-1] <= hi


# ---------------------------------------------------------------------------
# Chebyshev basis (Sec. 2, Definition): p_j = T_j(theta (M^{-1}A - sigma I)) p_0
# checked against T_j(cos phi) = cos(j phi) on the eigen-decomposition.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["poisson2d", "faces3d"])
def test_chebyshev_basis_closed_form(case):
    if case == "poisson2d":
        A = gen.poisson2d_csr(6, 5)
        lmin, lmax = gen.jacobi_poisson_bounds(6, 5)
    else:
        kx, ky, kz = gen.face_coefficients(gen.rng(2), 4, 3, 3, 0.5)
        A = oracle.assemble_stencil7(4, 3, 3, kx, ky, kz)
        lmin, lmax = gen.gershgorin_jacobi_bounds()
    Ad = dense(A)
    n = Ad.shape[0]
    invd, dv = oracle.jacobi(A)
    s = 12
    p0 = gen.uniform(gen.rng(5), n)
    P, AP = oracle.chebyshev_basis(A, invd, p0, s, lmin, lmax)
    # M^{-1} A = D^{-1/2} (V diag(lam) V^T) D^{1/2}
    dh = np.sqrt(dv)
    lam, V = np.linalg.eigh(Ad / dh[:, None] / dh[None, :])
    theta, sigma = 2 / (lmax - lmin), (lmax + lmin) / 2
    t = np.clip(theta * (lam - sigma), -1, 1)
    q = V.T @ (dh * p0)
    for j in range(s):
        pj = (V @ (np.cos(j * np.arccos(t)) * q)) / dh
        assert rel(P[j], pj) < 1e-12, j
        assert rel(AP[j], Ad @ P[j]) < 1e-14, j


# ---------------------------------------------------------------------------
# FGS (Sec. 2 / Sec. 3)
# ---------------------------------------------------------------------------

def synthetic_gram(s, seed, cond_shift=0.5):
    r = np.random.default_rng(seed)
    B = r.standard_normal((s + 3, s))
    H = B.T @ B + cond_shift * np.eye(s)
    dd = 1 / np.sqrt(np.diag(H))
    G = dd[:, None] * H * dd[None, :]
    np.fill_diagonal(G, 1.0)
    return G, r.standard_normal(s)


@pytest.mark.parametrize("s", [2, 5, 16, 32])
def test_fgs_converges_to_cholesky(s):
    """P2: with many sweeps FGS reaches the Cholesky solution of the SPD system."""
    G, c = synthetic_gram(s, s)
    Lc = np.linalg.cholesky(G)
    exact = np.linalg.solve(Lc.T, np.linalg.solve(Lc, c))
    a = oracle.fgs(G, c, 20000)
    assert rel(a, exact) < 1e-12


def test_fgs_two_by_two_closed_form():
    g, c0, c1 = 0.4, 1.3, -0.7
    G = np.array([[1.0, g], [g, 1.0]])
    a0, a1 = 0.0, 0.0
    for nu in range(1, 6):
        a0 = c0 - g * a1
        a1 = c1 - g * a0
        assert np.allclose(oracle.fgs(G, np.array([c0, c1]), nu), [a0, a1], rtol=0, atol=1e-15)


def test_fgs_identity_one_sweep():
    c = np.arange(1.0, 9.0)
    assert np.array_equal(oracle.fgs(np.eye(8), c, 1), c)


@pytest.mark.parametrize("s", [4, 16, 32])
def test_fgs_residual_structure(s):
    """P4 (Sec. 3, Proposition "FGS Residual Structure"):
    c - G a^{(l+1)} = L^T (a^{(l)} - a^{(l+1)}), and r^{(1)} = -L^T a^{(1)}."""
    G, c = synthetic_gram(s, 100 + s)
    LT = np.triu(G, 1)
    prev = np.zeros(s)
    for nu in range(1, 8):
        a = oracle.fgs(G, c, nu)
        lhs = c - G @ a
        rhs = LT @ (prev - a)
        assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(c)
        prev = a
    a1 = oracle.fgs(G, c, 1)
    assert np.linalg.norm((c - G @ a1) + LT @ a1) <= 1e-13 * np.linalg.norm(c)


def test_fgs_is_forward_not_backward():
    """A backward sweep would satisfy the identity with L instead of L^T; make
    sure the two differ on this example and the oracle matches the forward one."""
    G, c = synthetic_gram(6, 7)
    a1 = oracle.fgs(G, c, 1)
    assert np.linalg.norm((c - G @ a1) + np.triu(G, 1) @ a1) < 1e-14
    assert np.linalg.norm((c - G @ a1) + np.tril(G, -1) @ a1) > 1e-3


@pytest.mark.parametrize("s", [4, 16, 20])
def test_fgs_backward_stability(s):
    """P10 (Sec. 3, Theorem "Backward Stability"): the computed sweep solves
    (I + L) a^{(l+1)} = c - L^T a^{(l)} + dr with
    ||dr|| <= eps C(s) (||c|| + ||I+L|| ||a^{(l+1)}|| + ||L^T|| ||a^{(l)}||);
    the residual is recomputed in extended precision.  The last term accounts
    for the rounding of the right-hand side c - L^T a^{(l)}, which the sweep
    forms in the same accumulation."""
    G, c = synthetic_gram(s, 200 + s, cond_shift=0.05)
    L = np.tril(G, -1)
    ILl = (np.eye(s) + L).astype(np.longdouble)
    LTl = L.T.astype(np.longdouble)
    cl = c.astype(np.longdouble)
    prev = np.zeros(s)
    for nu in range(1, 6):
        a = oracle.fgs(G, c, nu)
        dr = ILl @ a.astype(np.longdouble) - (cl - LTl @ prev.astype(np.longdouble))
        bound = EPS * s * (np.linalg.norm(c) + np.linalg.norm(np.eye(s) + L, 2) * np.linalg.norm(a)
                           + np.linalg.norm(L.T, 2) * np.linalg.norm(prev))
        assert float(np.linalg.norm(dr.astype(np.float64))) <= bound
        prev = a


def test_fgs_g_norm_error_monotone():
    """Gauss-Seidel on an SPD matrix contracts the G-norm of the error at every
    sweep (Ostrowski-Reich), the valid form of the multi-sweep lemma (Sec. 3)."""
    G, c = synthetic_gram(16, 9, cond_shift=0.01)
    exact = np.linalg.solve(G, c)
    prev = np.inf
    for nu in range(0, 40):
        e = exact - oracle.fgs(G, c, nu) if nu else exact
        en = math.sqrt(e @ G @ e)
        assert en <= prev * (1 + 1e-12)
        prev = en


# ---------------------------------------------------------------------------
# Outer iteration (Sec. 2, Sec. 5, Sec. 7)
# ---------------------------------------------------------------------------

def small_problem(kind="poisson3d", seed=0):
    if kind == "poisson3d":
        pr = gen.small_poisson3d(6, 5, 4, seed=seed)
    elif kind == "faces3d":
        pr = gen.small_faces3d(5, 4, 4, seed=seed, sigma=1.0)
    else:
        r = gen.rng(seed)
        lmin, lmax = gen.jacobi_poisson_bounds(9, 7)
        pr = gen.Problem("p2d", "csr", (9, 7), 6, 25, lmin, lmax, xstar=gen.uniform(r, 63))
    A = oracle.problem_csr(pr)
    b = oracle.spmv(A, pr.xstar)
    return pr, A, b


@pytest.mark.parametrize("kind", ["poisson3d", "faces3d", "poisson2d"])
def test_gram_symmetric_spd_unit_diagonal(kind):
    """P5: G is exactly symmetric with unit diagonal and positive definite."""
    pr, A, b = small_problem(kind)
    out = oracle.step(A, b, np.zeros(pr.n), 6, 10, pr.lmin, pr.lmax)
    assert out["status"] == 0
    G = out["G"]
    assert np.array_equal(G, G.T) and np.array_equal(out["Graw"], out["Graw"].T)
    assert np.all(np.diag(G) == 1.0)
    np.linalg.cholesky(G)


@pytest.mark.parametrize("kind", ["poisson3d", "faces3d", "poisson2d"])
@pytest.mark.parametrize("p0_mode", [0, 1])
def test_one_sweep_equals_a_norm_mgs(kind, p0_mode):
    """P3 (Sec. 5, Theorem "Algebraic Equivalence"): one FGS sweep from zero on
    G a = P~^T A e, with e = x* - x_k (so that P~^T A e = P~^T r_k), gives the
    coefficients of one A-norm MGS pass of e against the scaled basis."""
    pr, A, b = small_problem(kind, seed=1)
    Ad = dense(A)
    xk = 0.3 * gen.uniform(gen.rng(11), pr.n)
    out = oracle.step(A, b, xk, 5, 1, pr.lmin, pr.lmax, p0_mode=p0_mode, want_basis=True)
    Pt = out["P"] * out["d"][:, None]
    w = pr.xstar - xk
    gam = np.zeros(5)
    for j in range(5):
        gam[j] = w @ (Ad @ Pt[j])
        w = w - gam[j] * Pt[j]
    assert rel(out["atil"], gam) < 1e-12
    # and the scaled right-hand side is P~^T r_k
    assert rel(out["ctil"], Pt @ (b - Ad @ xk)) < 1e-13


@pytest.mark.parametrize("kind", ["poisson3d", "faces3d"])
def test_energy_identity_each_outer(kind):
    """P6: ||e_{k+1}||_A^2 - ||e_k||_A^2 = atil^T G atil - 2 ctil^T atil <= 0,
    the A-norm error never grows even with an inexact Gram solve."""
    pr, A, b = small_problem(kind, seed=2)
    Ad = dense(A)
    x = np.zeros(pr.n)
    for _ in range(6):
        out = oracle.step(A, b, x, 6, 3, pr.lmin, pr.lmax)
        e0 = pr.xstar - x
        e1 = pr.xstar - out["x"]
        lhs = e1 @ Ad @ e1 - e0 @ Ad @ e0
        a, G, c = out["atil"], out["G"], out["ctil"]
        rhs = a @ G @ a - 2 * c @ a
        assert rhs <= 0
        assert abs(lhs - rhs) <= 1e-11 * (e0 @ Ad @ e0)
        x = out["x"]


def test_s1_is_preconditioned_steepest_descent():
    """P7: with s = 1 the update is x + (z^T r / z^T A z) z, z = M^{-1} r."""
    pr, A, b = small_problem("faces3d", seed=4)
    Ad = dense(A)
    xk = 0.1 * gen.uniform(gen.rng(1), pr.n)
    r = b - Ad @ xk
    z = r / np.diag(Ad)
    want = xk + (z @ r) / (z @ Ad @ z) * z
    out = oracle.step(A, b, xk, 1, 7, pr.lmin, pr.lmax)
    assert rel(out["x"], want) < 1e-14


def test_exact_gram_solve_gives_galerkin_orthogonality():
    """P8: with enough sweeps the new residual is orthogonal to the basis."""
    pr, A, b = small_problem("poisson3d", seed=3)
    Ad = dense(A)
    xk = np.zeros(pr.n)
    out = oracle.step(A, b, xk, 4, 20000, pr.lmin, pr.lmax, want_basis=True)
    Pt = out["P"] * out["d"][:, None]
    r1 = b - Ad @ out["x"]
    assert np.linalg.norm(Pt @ r1) <= 1e-10 * np.linalg.norm(out["ctil"])


@pytest.mark.parametrize("dims,s", [((8, 8), 4), ((8, 8), 8), ((6, 6, 6), 4), ((6, 6, 6), 8)])
def test_converges_to_dense_direct_solve(dims, s):
    """P9: tight tolerance reaches the direct solution within kappa(A) * tol."""
    r = gen.rng(7)
    A = gen.poisson2d_csr(*dims) if len(dims) == 2 else gen.poisson3d_csr(*dims)
    lmin, lmax = gen.jacobi_poisson_bounds(*dims)
    n = int(np.prod(dims))
    b = gen.uniform(r, n)
    out = oracle.solve(A, b, None, s, 25, lmin, lmax, 1e-12)
    assert out["status"] == 0
    Ad = dense(A)
    xs = np.linalg.solve(Ad, b)
    assert rel(out["x"], xs) <= np.linalg.cond(Ad) * 1e-12


def test_stencil_and_csr_forms_agree():
    """P13: the oracle's stencil assembly and the generator's CSR of the same
    face operator give the same outer iteration."""
    pr = gen.small_faces3d(6, 5, 4, seed=8)
    A1 = oracle.problem_csr(pr)
    A2 = pr.csr()
    b = oracle.spmv(A1, pr.xstar)
    o1 = oracle.step(A1, b, np.zeros(pr.n), 8, 25, pr.lmin, pr.lmax)
    o2 = oracle.step(A2, b, np.zeros(pr.n), 8, 25, pr.lmin, pr.lmax)
    assert rel(o1["atil"], o2["atil"]) < 1e-12 and rel(o1["x"], o2["x"]) < 1e-12


def test_p0_modes_identical_for_constant_diagonal():
    """With a constant Jacobi diagonal, p_0 = M^{-1} r and p_0 = r differ by a
    scalar that the column scaling absorbs: same scaled coefficients."""
    pr, A, b = small_problem("poisson3d", seed=5)
    o0 = oracle.step(A, b, np.zeros(pr.n), 8, 25, pr.lmin, pr.lmax, p0_mode=0)
    o1 = oracle.step(A, b, np.zeros(pr.n), 8, 25, pr.lmin, pr.lmax, p0_mode=1)
    assert rel(o0["atil"], o1["atil"]) < 1e-12 and rel(o0["x"], o1["x"]) < 1e-12


# ---------------------------------------------------------------------------
# Solve loop: stopping rule and failure paths
# ---------------------------------------------------------------------------

def test_stopping_rule_strict_and_counts():
    pr = gen.config1()
    A = pr.csr()
    b = oracle.spmv(A, pr.xstar)
    out = oracle.solve(A, b, None, pr.s, pr.nu, pr.lmin, pr.lmax, 1e-8, hist_cap=1000)
    k = out["iters"]
    h = out["hist_relres"]
    assert out["status"] == 0 and h[k] < 1e-8 and np.all(h[:k] >= 1e-8) and h[0] == 1.0
    assert abs(out["relres"] - h[k]) == 0
    # the reported residual is the true one of the returned x
    assert abs(np.linalg.norm(b - oracle.spmv(A, out["x"])) / np.linalg.norm(b) - out["relres"]) < 1e-12


def test_zero_rhs_returns_immediately():
    A = gen.poisson2d_csr(5, 5)
    out = oracle.solve(A, np.zeros(25), None, 4, 5, *gen.jacobi_poisson_bounds(5, 5), 1e-8)
    assert out["status"] == 0 and out["iters"] == 0 and np.all(out["x"] == 0)


def test_max_outer_gives_noconv_with_last_iterate():
    pr = gen.config1()
    A = pr.csr()
    b = oracle.spmv(A, pr.xstar)
    out = oracle.solve(A, b, None, pr.s, pr.nu, pr.lmin, pr.lmax, 1e-8, max_outer=3)
    assert out["status"] == 5 and out["iters"] == 3
    x = np.zeros(pr.n)
    for _ in range(3):
        x = oracle.step(A, b, x, pr.s, pr.nu, pr.lmin, pr.lmax)["x"]
    assert np.array_equal(x, out["x"])


def test_breakdown_when_basis_vector_vanishes():
    """A = 2I, no preconditioner, bounds [1, 3] -> sigma = 2, so p_1 = 0 exactly
    and p_1^T A p_1 = 0: the column scaling is undefined."""
    n = 10
    A = (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.full(n, 2.0))
    out = oracle.solve(A, np.ones(n), None, 3, 5, 1.0, 3.0, 1e-8, precond=0)
    assert out["status"] == 4 and out["iters"] == 0 and np.all(out["x"] == 0)


def test_nonfinite_rhs():
    A = gen.poisson2d_csr(5, 5)
    b = np.ones(25)
    b[3] = np.nan
    out = oracle.solve(A, b, None, 4, 5, *gen.jacobi_poisson_bounds(5, 5), 1e-8)
    assert out["status"] == 6


@pytest.mark.parametrize("bad", ["s0", "nu0", "bounds", "tol", "csr"])
def test_argument_errors(bad):
    A = gen.poisson2d_csr(4, 4)
    args = dict(s=4, nu=5, lmin=0.1, lmax=1.9, tol=1e-8)
    if bad == "s0":
        args["s"] = 0
    elif bad == "nu0":
        args["nu"] = 0
    elif bad == "bounds":
        args["lmin"], args["lmax"] = 1.9, 0.1
    elif bad == "tol":
        args["tol"] = 1.5
    else:
        rp, ci, v = A
        ci = ci.copy()
        ci[3] = 99
        A = (rp, ci, v)
    out = oracle.solve(A, np.ones(16), None, args["s"], args["nu"], args["lmin"], args["lmax"], args["tol"])
    assert out["status"] == 1


# ---------------------------------------------------------------------------
# P11: gradient through the solve (adjoint), against complex-step derivatives
# of a dense direct solve (exact to rounding, no finite-difference error)
# ---------------------------------------------------------------------------

def dense_faces(nx, ny, nz, kx, ky, kz):
    """Dense face operator built from its definition, complex-safe."""
    n = nx * ny * nz
    M = np.zeros((n, n), dtype=np.result_type(kx, ky, kz))
    KX = kx.reshape(nz, ny, nx + 1)
    KY = ky.reshape(nz, ny + 1, nx)
    KZ = kz.reshape(nz + 1, ny, nx)
    idx = lambda i, j, k: i + nx * (j + ny * k)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                p = idx(i, j, k)
                for kf, q in [(KX[k, j, i], idx(i - 1, j, k) if i > 0 else None),
                              (KX[k, j, i + 1], idx(i + 1, j, k) if i < nx - 1 else None),
                              (KY[k, j, i], idx(i, j - 1, k) if j > 0 else None),
                              (KY[k, j + 1, i], idx(i, j + 1, k) if j < ny - 1 else None),
                              (KZ[k, j, i], idx(i, j, k - 1) if k > 0 else None),
                              (KZ[k + 1, j, i], idx(i, j, k + 1) if k < nz - 1 else None)]:
                    M[p, p] += kf
                    if q is not None:
                        M[p, q] -= kf
    return M


def test_gradient_faces_matches_complex_step():
    nx, ny, nz = 4, 3, 3
    r = gen.rng(12)
    kx, ky, kz = gen.face_coefficients(r, nx, ny, nz, 0.5)
    n = nx * ny * nz
    b = gen.uniform(r, n)
    xt = gen.uniform(r, n)

    def loss(kx_, ky_, kz_, b_):
        x = np.linalg.solve(dense_faces(nx, ny, nz, kx_, ky_, kz_), b_)
        return 0.5 * np.sum((x - xt) ** 2)

    A = oracle.assemble_stencil7(nx, ny, nz, kx, ky, kz)
    assert np.allclose(dense(A), dense_faces(nx, ny, nz, kx, ky, kz), rtol=0, atol=1e-15)
    lmin, lmax = gen.gershgorin_jacobi_bounds()
    fwd = oracle.solve(A, b, None, 8, 25, lmin, lmax, 1e-13)
    x = fwd["x"]
    adj = oracle.solve(A, x - xt, None, 8, 25, lmin, lmax, 1e-13)
    lam = adj["x"]
    assert fwd["status"] == 0 and adj["status"] == 0
    gx, gy, gz = oracle.grad_faces(nx, ny, nz, lam, x)
    h = 1e-30
    scale = max(np.abs(gx).max(), np.abs(gy).max(), np.abs(gz).max())
    for arr, g, which in [(kx, gx, 0), (ky, gy, 1), (kz, gz, 2)]:
        for f in range(arr.size):
            kk = [kx.astype(complex), ky.astype(complex), kz.astype(complex)]
            kk[which][f] += 1j * h
            cs = loss(*kk, b.astype(complex)).imag / h
            assert abs(cs - g[f]) <= 1e-9 * scale, (which, f)
    for m in range(n):
        bb = b.astype(complex)
        bb[m] += 1j * h
        cs = loss(kx, ky, kz, bb).imag / h
        assert abs(cs - lam[m]) <= 1e-9 * np.abs(lam).max()


def test_gradient_csr_matches_complex_step():
    A = gen.poisson2d_csr(4, 4)
    rp, ci, v = A
    r = gen.rng(13)
    b = gen.uniform(r, 16)
    xt = gen.uniform(r, 16)
    lmin, lmax = gen.jacobi_poisson_bounds(4, 4)
    x = oracle.solve(A, b, None, 4, 25, lmin, lmax, 1e-13)["x"]
    lam = oracle.solve(A, x - xt, None, 4, 25, lmin, lmax, 1e-13)["x"]
    g = oracle.grad_csr(A, lam, x)
    h = 1e-30
    for k in range(v.size):
        vals = v.astype(complex)
        vals[k] += 1j * h
        M = np.zeros((16, 16), complex)
        for i in range(16):
            M[i, ci[rp[i]:rp[i + 1]]] = vals[rp[i]:rp[i + 1]]
        cs = (0.5 * np.sum((np.linalg.solve(M, b) - xt) ** 2)).imag / h
        assert abs(cs - g[k]) <= 1e-9 * np.abs(g).max(), k


def test_golden_c1_trajectory_unchanged():
    """Regression fixture written by tests/golden/make_golden.py (oracle only)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "c1_oracle.json")) as f:
        g = json.load(f)
    pr = gen.config1(0)
    A = pr.csr()
    b = oracle.spmv(A, pr.xstar)
    out = oracle.solve(A, b, None, pr.s, pr.nu, pr.lmin, pr.lmax, pr.tol, hist_cap=1000)
    assert out["iters"] == g["iters"]
    assert np.allclose(out["hist_relres"], g["hist_relres"], rtol=1e-12, atol=0)
    first = oracle.step(A, b, np.zeros(pr.n), pr.s, pr.nu, pr.lmin, pr.lmax)
    assert np.allclose(first["atil"], g["atil_first"], rtol=1e-13, atol=0)
    assert (g["lmin"], g["lmax"]) == (pr.lmin, pr.lmax)


# ---------------------------------------------------------------------------
# Gram diagnostics: delta_k (Sec. 7), ||L||_F (Sec. 4), kappa(G) (Sec. 4, 8)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["poisson3d", "faces3d", "poisson2d"])
@pytest.mark.parametrize("nu", [1, 2, 7])
def test_delta_is_residual_structure_of_last_sweep(kind, nu):
    """delta_k = ||ctil - G atil|| / ||ctil|| must equal, by the FGS residual
    structure (Sec. 3, Proposition), ||L^T (atil^(nu-1) - atil^(nu))|| / ||ctil||
    with atil^(0) = 0: at nu = 1 that is ||L^T atil^(1)|| / ||ctil||.  The two
    sweep counts come from the oracle's FGS; the step's own delta is computed
    as a residual, so a dropped term, G_raw in place of G or the wrong
    denominator in either breaks the equality."""
    pr, A, b = small_problem(kind, seed=5)
    out = oracle.step(A, b, np.zeros(pr.n), 6, nu, pr.lmin, pr.lmax)
    assert out["status"] == 0
    G, ct = out["G"], out["ctil"]
    L = np.tril(G, -1)
    prev = oracle.fgs(G, ct, nu - 1) if nu > 1 else np.zeros(6)
    last = oracle.fgs(G, ct, nu)
    assert np.array_equal(last, out["atil"])
    want = np.linalg.norm(L.T @ (prev - last)) / np.linalg.norm(ct)
    assert abs(out["delta"] - want) <= 1e-13 * max(want, 1e-3), (out["delta"], want)
    assert out["delta"] > 0


@pytest.mark.parametrize("kind", ["poisson3d", "faces3d", "poisson2d"])
def test_lnorm_from_frobenius_identity(kind):
    """||L||_F with G = I + L + L^T (Sec. 4): ||G||_F^2 = s + 2 ||L||_F^2, an
    identity independent of how L is read off G; the solve's per-update history
    equals the step's value at the same iterate."""
    pr, A, b = small_problem(kind, seed=6)
    s = 6
    out = oracle.step(A, b, np.zeros(pr.n), s, 10, pr.lmin, pr.lmax)
    G = out["G"]
    want = math.sqrt((np.sum(G * G) - s) / 2)
    assert abs(out["lnorm"] - want) <= 1e-13 * want
    sol = oracle.solve(A, b, None, s, 10, pr.lmin, pr.lmax, 1e-10, hist_cap=200)
    assert sol["hist_lnorm"][0] == out["lnorm"]
    assert sol["hist_delta"][0] == out["delta"]


def test_lnorm_grows_like_sqrt_s():
    """Sec. 4, Theorem "Polynomial Growth": with column scaling the Chebyshev
    Gram matrix has ||L||_F = O(sqrt(s)).  On an operator whose spectrum fills
    the Chebyshev interval [0, 2] (a diagonal matrix, no preconditioner, so the
    bounds are exact) ||L||_F^2 / s must stay bounded and flat as s grows from
    4 to 32 (the monomial basis would grow exponentially)."""
    n = 4000
    lam = np.linspace(0.0, 2.0, n + 2)[1:-1]
    A = (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), lam.copy())
    ratios = []
    for s in (4, 8, 16, 32):
        out = oracle.step(A, np.ones(n), np.zeros(n), s, 5, 0.0, 2.0, precond=0)
        assert out["status"] == 0
        ratios.append(out["lnorm"] ** 2 / s)
    assert max(ratios) <= 0.5, ratios
    assert max(ratios) / min(ratios) <= 1.2, ratios


def test_gram_condition_closed_form():
    """kappa of the tridiagonal Toeplitz matrix I + a (E + E^T), whose
    eigenvalues are 1 + 2a cos(k pi / (s + 1)), k = 1..s (textbook)."""
    for s, a in [(5, 0.3), (16, 0.45), (32, -0.2)]:
        G = np.eye(s) + a * (np.eye(s, k=1) + np.eye(s, k=-1))
        ev = 1 + 2 * a * np.cos(np.arange(1, s + 1) * math.pi / (s + 1))
        want = ev.max() / ev.min()
        assert abs(oracle.gram_condition(G) - want) <= 1e-12 * want
    assert oracle.gram_condition(np.array([[1.0, 1.0], [1.0, 1.0]])) == float("inf") or \
        oracle.gram_condition(np.array([[1.0, 1.0], [1.0, 1.0]])) > 1e15


# ---------------------------------------------------------------------------
# Lanczos spectrum bounds (Sec. 8 setup)
# ---------------------------------------------------------------------------

def _krylov_ritz(Ad, d, u, m):
    """Rayleigh-Ritz values of M^{-1}A on K_m(M^{-1}A, u), computed densely:
    B = D^{-1/2} A D^{-1/2} on an orthonormal (QR) basis of D^{1/2} K_m."""
    s = np.sqrt(d)
    B = Ad / s[:, None] / s[None, :]
    K = np.zeros((u.size, m))
    v = s * u
    for j in range(m):
        K[:, j] = v / np.linalg.norm(v)
        v = B @ K[:, j]
    Q, _ = np.linalg.qr(K)
    return np.linalg.eigvalsh(Q.T @ B @ Q)


@pytest.mark.parametrize("kind", ["poisson3d", "faces3d", "poisson2d"])
def test_lanczos_ritz_values_are_krylov_projection(kind):
    """The Ritz values of a few Lanczos steps are the eigenvalues of M^{-1}A
    projected on the Krylov space K_m(M^{-1}A, u) (textbook Rayleigh-Ritz),
    formed here densely from a QR of the Krylov basis."""
    pr, A, _ = small_problem(kind, seed=7)
    Ad = dense(A)
    d = np.diag(Ad).copy()
    u = gen.uniform(gen.rng(3), pr.n)
    for m in (2, 5, 8):
        out = oracle.lanczos(A, u, m)
        assert out["m"] == m
        want = _krylov_ritz(Ad, d, u, m)
        assert np.max(np.abs(out["ritz"] - want)) <= 1e-10 * np.abs(want).max(), (m, out["ritz"], want)


@pytest.mark.parametrize("dims", [(3, 3, 2), (4, 3, 3)])
def test_lanczos_full_run_finds_exact_extremes(dims):
    """With as many steps as unknowns the extreme Ritz values reach the closed-
    form extreme eigenvalues of the Jacobi-preconditioned Poisson operator."""
    nx, ny, nz = dims
    A = oracle.assemble_stencil7(nx, ny, nz)
    n = nx * ny * nz
    lo, hi = gen.jacobi_poisson_bounds(nx, ny, nz)
    out = oracle.lanczos(A, gen.uniform(gen.rng(1), n), n)
    assert abs(out["ritz"][0] - lo) <= 1e-10 and abs(out["ritz"][-1] - hi) <= 1e-10, (out["ritz"], lo, hi)


def test_lanczos_ten_steps_inside_spectrum_and_margin():
    """Ten steps on 20^3 Poisson: every Ritz value lies inside the exact
    spectrum of M^{-1}A (Cauchy interlacing), the largest is already close to
    lambda_max, and the 10% margin widens the extremes as stated."""
    N = 20
    A = oracle.assemble_stencil7(N, N, N)
    lo, hi = gen.jacobi_poisson_bounds(N, N, N)
    out = oracle.lanczos(A, gen.uniform(gen.rng(2), N ** 3), 10)
    r = out["ritz"]
    assert out["m"] == 10 and r.size == 10
    assert r[0] >= lo - 1e-12 and r[-1] <= hi + 1e-12
    assert hi - r[-1] <= 0.05 * hi
    bl, bh = oracle.lanczos_bounds(r, 0.1)
    assert bl == 0.9 * r[0] and bh == 1.1 * r[-1]
    assert bh > hi


def test_lanczos_faces_inside_gershgorin_and_dense_spectrum():
    pr, A, _ = small_problem("faces3d", seed=8)
    Ad = dense(A)
    d = np.diag(Ad)
    ev = np.linalg.eigvalsh(Ad / np.sqrt(d)[:, None] / np.sqrt(d)[None, :])
    out = oracle.lanczos(A, gen.uniform(gen.rng(4), pr.n), 10)
    assert out["ritz"][0] >= ev[0] - 1e-12 and out["ritz"][-1] <= ev[-1] + 1e-12
    assert 0.0 <= out["ritz"][0] and out["ritz"][-1] <= 2.0


def test_lanczos_stops_on_invariant_subspace_and_zero_start():
    """An eigenvector start spans an invariant subspace: one step, Ritz value
    = its eigenvalue; a zero start vector gives no steps."""
    nx, ny, nz = 5, 4, 3
    A = oracle.assemble_stencil7(nx, ny, nz)
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    k = np.arange(nz)[:, None, None]
    v = (np.sin(math.pi * (i + 1) / (nx + 1)) * np.sin(2 * math.pi * (j + 1) / (ny + 1))
         * np.sin(math.pi * (k + 1) / (nz + 1))).ravel()
    lam = (6 - 2 * math.cos(math.pi / (nx + 1)) - 2 * math.cos(2 * math.pi / (ny + 1))
           - 2 * math.cos(math.pi / (nz + 1))) / 6
    out = oracle.lanczos(A, v, 10)
    assert out["m"] == 1 and abs(out["ritz"][0] - lam) <= 1e-14
    assert oracle.lanczos(A, np.zeros(nx * ny * nz), 10)["m"] == 0


# ---------------------------------------------------------------------------
# The 27-point operator of the paper's experiments (Sec. 8)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dims", [(5, 4, 3), (9, 9, 9)])
def test_poisson27_sine_eigenpairs(dims):
    """A = 27 I - T_x (x) T_y (x) T_z: sine eigenvectors with eigenvalues
    27 - prod_a (1 + 2 cos(m_a pi / (N_a + 1))); the generator's CSR and the
    oracle's assembly are the same matrix."""
    nx, ny, nz = dims
    Ao = oracle.assemble_stencil27(nx, ny, nz)
    Ag = gen.poisson27_csr(nx, ny, nz)
    for a, b in zip(Ao, Ag):
        assert np.array_equal(a, b)
    rp, ci, v = Ao
    assert rp[-1] == (3 * nx - 2) * (3 * ny - 2) * (3 * nz - 2)
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    k = np.arange(nz)[:, None, None]
    for a, b, c in [(1, 1, 1), (2, 3, 1), (nx, ny, nz), (nx, 1, 1), (1, ny, 2)]:
        vec = (np.sin(a * math.pi * (i + 1) / (nx + 1)) * np.sin(b * math.pi * (j + 1) / (ny + 1))
               * np.sin(c * math.pi * (k + 1) / (nz + 1))).ravel()
        lam = 27 - ((1 + 2 * math.cos(a * math.pi / (nx + 1))) * (1 + 2 * math.cos(b * math.pi / (ny + 1)))
                    * (1 + 2 * math.cos(c * math.pi / (nz + 1))))
        assert np.linalg.norm(oracle.spmv(Ao, vec) - lam * vec) < 54 * 1e-14 * np.linalg.norm(vec)


@pytest.mark.parametrize("dims", [(5, 4, 3), (8, 8, 8), (11, 6, 9)])
def test_poisson27_jacobi_bounds_closed_form(dims):
    """The corner rule of the bounds equals the dense spectrum of D^{-1} A."""
    nx, ny, nz = dims
    Ad = dense(oracle.assemble_stencil27(nx, ny, nz))
    ev = np.linalg.eigvalsh(Ad / 26.0)
    lo, hi = gen.jacobi_poisson27_bounds(nx, ny, nz)
    assert abs(ev[0] - lo) <= 1e-13 and abs(ev[-1] - hi) <= 1e-13, (ev[0], lo, ev[-1], hi)


def test_poisson27_solve_converges_to_direct_solution():
    """P9 on the 27-point operator: the s-step solve at tol 1e-12 reaches the
    dense direct solution within kappa(A) tol."""
    pr = gen.small_poisson27(7, 6, 5, seed=3, s=8, nu=30)
    A = oracle.problem_csr(pr)
    b = oracle.spmv(A, pr.xstar)
    out = oracle.solve(A, b, None, pr.s, pr.nu, pr.lmin, pr.lmax, 1e-12)
    assert out["status"] == 0
    Ad = dense(A)
    ev = np.linalg.eigvalsh(Ad)
    xd = np.linalg.solve(Ad, b)
    assert rel(out["x"], xd) <= (ev[-1] / ev[0]) * 1e-12


# ---------------------------------------------------------------------------
# Monomial basis (the comparison of Sec. 4)
# ---------------------------------------------------------------------------

def test_monomial_basis_closed_form_on_eigenvector():
    """p_j = (M^{-1}A)^j p_0: on an eigenvector v of M^{-1}A with eigenvalue
    lambda the basis is lambda^j v and A p_j = 6 lambda^{j+1} v (Poisson)."""
    nx, ny, nz = 6, 5, 4
    A = oracle.assemble_stencil7(nx, ny, nz)
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    k = np.arange(nz)[:, None, None]
    v = (np.sin(2 * math.pi * (i + 1) / (nx + 1)) * np.sin(math.pi * (j + 1) / (ny + 1))
         * np.sin(3 * math.pi * (k + 1) / (nz + 1))).ravel()
    lam = (6 - 2 * math.cos(2 * math.pi / (nx + 1)) - 2 * math.cos(math.pi / (ny + 1))
           - 2 * math.cos(3 * math.pi / (nz + 1))) / 6
    b = oracle.spmv(A, v)  # r_0 = b for x_0 = 0, p_0 = M^{-1} r_0 = lambda v
    out = oracle.step(A, b, np.zeros(v.size), 5, 3, 0.1, 1.9, want_basis=True, basis="monomial")
    for jj in range(5):
        assert np.linalg.norm(out["P"][jj] - lam ** (jj + 1) * v) <= 1e-13 * np.linalg.norm(v)
        assert np.linalg.norm(out["AP"][jj] - 6 * lam ** (jj + 2) * v) <= 1e-12 * np.linalg.norm(v)


def test_monomial_gram_condition_grows_exponentially():
    """Sec. 4, monomial comparison: the column-scaled monomial Gram matrix is
    far worse conditioned than the Chebyshev one, and its condition grows
    much faster with s."""
    N = 16
    A = oracle.assemble_stencil7(N, N, N)
    lo, hi = gen.jacobi_poisson_bounds(N, N, N)
    b = oracle.spmv(A, gen.uniform(gen.rng(8), N ** 3))
    kc, km = {}, {}
    for s in (4, 6, 8):
        oc = oracle.step(A, b, np.zeros(N ** 3), s, 5, lo, hi)
        om = oracle.step(A, b, np.zeros(N ** 3), s, 5, lo, hi, basis="monomial")
        kc[s], km[s] = oracle.gram_condition(oc["G"]), oracle.gram_condition(om["G"])
    assert km[8] > 1e4 * kc[8], (kc, km)
    # per two more columns the monomial condition grows >= 100x and at least
    # 10x faster than the Chebyshev one
    for s0 in (4, 6):
        gm, gc = km[s0 + 2] / km[s0], kc[s0 + 2] / kc[s0]
        assert gm >= 100 and gm >= 10 * gc, (s0, gm, gc)


# ---------------------------------------------------------------------------
# Two-level hierarchy and the coarse FGS solve (Sec. 6; Sec. 8)
# ---------------------------------------------------------------------------

def _face_energy(nx, ny, nz, kx, ky, kz, v):
    """sum over faces of k_f (v_p - v_q)^2, v = 0 outside (Dirichlet)."""
    V = np.zeros((nz + 2, ny + 2, nx + 2))
    V[1:-1, 1:-1, 1:-1] = v.reshape(nz, ny, nx)
    kx = kx.reshape(nz, ny, nx + 1)
    ky = ky.reshape(nz, ny + 1, nx)
    kz = kz.reshape(nz + 1, ny, nx)
    ex = np.sum(kx * (V[1:-1, 1:-1, 1:] - V[1:-1, 1:-1, :-1]) ** 2)
    ey = np.sum(ky * (V[1:-1, 1:, 1:-1] - V[1:-1, :-1, 1:-1]) ** 2)
    ez = np.sum(kz * (V[1:, 1:-1, 1:-1] - V[:-1, 1:-1, 1:-1]) ** 2)
    return ex + ey + ez


@pytest.mark.parametrize("nc", [(3, 2, 4), (5, 5, 5)])
def test_prolongation_row_and_column_sums(nc):
    """Trilinear hats: every coarse column sums to (1/2 + 1 + 1/2)^3 = 8 and
    carries 27 entries; P 1 = 1 at fine points off the boundary layer, and
    1/2 per axis on which the point lies next to the boundary."""
    rp, ci, v = oracle.prolongation(*nc)
    nf = [2 * c + 1 for c in nc]
    n_f, n_c = int(np.prod(nf)), int(np.prod(nc))
    assert rp.size == n_f + 1
    colsum = np.bincount(ci, weights=v, minlength=n_c)
    assert np.all(colsum == 8.0) and np.all(np.bincount(ci, minlength=n_c) == 27)
    ones = np.add.reduceat(v, rp[:-1]) * (np.diff(rp) > 0)
    want = np.ones(nf[::-1])
    for axis, n in zip((2, 1, 0), nf):
        sl = [slice(None)] * 3
        for edge in (0, n - 1):
            sl[axis] = edge
            want[tuple(sl)] *= 0.5
    assert np.array_equal(ones, want.ravel())


@pytest.mark.parametrize("seed", [0, 1])
def test_galerkin_energy_identity(seed):
    """u^T A_c u = (P u)^T A_f (P u) = sum_f k_f ((Pu)_p - (Pu)_q)^2 (the face
    energy, computed from P u alone); A_c is symmetric positive definite with
    the 27-point coarse pattern."""
    tl = gen.two_level(seed, nc=(4, 3, 5), sigma=1.0)
    nx, ny, nz = tl.nf
    P = oracle.prolongation(*tl.nc)
    Af = oracle.assemble_stencil7(nx, ny, nz, tl.kx, tl.ky, tl.kz)
    Ac = oracle.galerkin(Af, P, tl.n_coarse)
    D = dense(Ac)
    assert np.array_equal(D, D.T) or np.max(np.abs(D - D.T)) <= 1e-14 * np.abs(D).max()
    np.linalg.cholesky(D)
    assert Ac[0][-1] == (3 * 4 - 2) * (3 * 3 - 2) * (3 * 5 - 2)
    Pd = np.zeros((nx * ny * nz, tl.n_coarse))
    for r in range(nx * ny * nz):
        Pd[r, P[1][P[0][r]:P[0][r + 1]]] = P[2][P[0][r]:P[0][r + 1]]
    for k in range(3):
        u = gen.uniform(gen.rng(10 + k), tl.n_coarse)
        e = _face_energy(nx, ny, nz, tl.kx, tl.ky, tl.kz, Pd @ u)
        assert abs(u @ D @ u - e) <= 1e-12 * e


def test_gs_converges_and_descends():
    """Forward GS is coordinate descent on E(u) = u^T A u / 2 - f^T u: E never
    grows from one sweep to the next, and many sweeps reach the dense direct
    solution of the coarse system."""
    tl = gen.two_level(2, nc=(5, 4, 3), sigma=0.5)
    u, Ac = oracle.coarse_fgs(tl.nc, tl.kx, tl.ky, tl.kz, tl.f, 1)
    D = dense(Ac)
    energy = [0.0]
    for nu in range(1, 8):
        u = oracle.gs(Ac, tl.f, nu)
        energy.append(0.5 * u @ D @ u - tl.f @ u)
    assert all(b <= a + 1e-14 for a, b in zip(energy, energy[1:])), energy
    u = oracle.gs(Ac, tl.f, 3000)
    assert rel(u, np.linalg.solve(D, tl.f)) <= 1e-10


def test_gs_two_by_two_closed_form():
    """One sweep on [[a, b], [b, c]]: u0 = f0 / a, u1 = (f1 - b u0) / c."""
    A = (np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32), np.array([4.0, -1.5, -1.5, 3.0]))
    f = np.array([2.0, 1.0])
    u = oracle.gs(A, f, 1)
    assert u[0] == 0.5 and u[1] == (1.0 + 1.5 * 0.5) / 3.0
