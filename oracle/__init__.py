"""FP64 CPU oracle of the s-step CG outer iteration with FGS Gram solves.

TEST INFRASTRUCTURE -- NOT PART OF THE PRODUCT.  Only ``tests/``, the smoke
check and the CPU-baseline leg of the benchmark may import this package.  It
wraps ``oracle.c`` (plain loops, FP64, compensated reductions) through ctypes
with NumPy arrays, and shares nothing with the HIP library.

Parity pins (see ``tests/test_oracle_pins.py``) tie every function here to
closed forms, invariants or theorems of the paper rather than to itself.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, LIB_OMP, build

_lib = None
_libs = {}

STATUS = {0: "OK", 1: "E_ARG", 3: "E_NOMEM", 4: "E_BREAKDOWN", 5: "E_NOCONV", 6: "E_NONFINITE"}


def select_build(openmp: bool) -> int:
    """Route every function of this module to the sequential reference build
    (default, the one the tests pin) or to the OpenMP timing build of the same
    source (CPU baseline only).  Returns the OpenMP thread count in use (1 for
    the reference build)."""
    global _lib
    _lib = None
    lib = _load(LIB_OMP if openmp else LIB)
    if not openmp:
        return 1
    f = lib.omp_get_max_threads
    f.restype = C.c_int
    return int(f())


def _load(path=None):
    global _lib
    if path is None and _lib is not None:
        return _lib
    # a sanitizer build of the same source, for the instrumented test run
    path = path or os.environ.get("SSTEP_ORACLE_LIB") or LIB
    if path in _libs:
        _lib = _libs[path]
        return _lib
    if not os.path.exists(path):
        build()
    _lib = C.CDLL(path)
    _libs[path] = _lib
    d, i32, i64 = C.c_double, C.c_int32, C.c_int64
    pd, pi = C.POINTER(C.c_double), C.POINTER(C.c_int32)
    _lib.oracle_dot.restype = d
    _lib.oracle_dot.argtypes = [i64, pd, pd]
    _lib.oracle_csr_validate.restype = C.c_int
    _lib.oracle_csr_validate.argtypes = [i64, pi, pi]
    _lib.oracle_spmv.restype = None
    _lib.oracle_spmv.argtypes = [i64, pi, pi, pd, pd, pd]
    _lib.oracle_stencil7_nnz.restype = i64
    _lib.oracle_stencil7_nnz.argtypes = [i32, i32, i32]
    _lib.oracle_assemble_stencil7.restype = i64
    _lib.oracle_assemble_stencil7.argtypes = [i32, i32, i32, pd, pd, pd, pi, pi, pd]
    _lib.oracle_stencil27_nnz.restype = i64
    _lib.oracle_stencil27_nnz.argtypes = [i32, i32, i32]
    _lib.oracle_assemble_stencil27.restype = i64
    _lib.oracle_assemble_stencil27.argtypes = [i32, i32, i32, pi, pi, pd]
    _lib.oracle_jacobi.restype = C.c_int
    _lib.oracle_jacobi.argtypes = [i64, pi, pi, pd, C.c_int, pd, pd]
    _lib.oracle_chebyshev_basis.restype = None
    _lib.oracle_chebyshev_basis.argtypes = [i64, pi, pi, pd, pd, C.c_int, d, d, pd, pd]
    _lib.oracle_gram.restype = None
    _lib.oracle_gram.argtypes = [i64, C.c_int, pd, pd, pd, pd, pd]
    _lib.oracle_column_scale.restype = C.c_int
    _lib.oracle_column_scale.argtypes = [C.c_int, pd, pd, pd, pd, pd]
    _lib.oracle_fgs.restype = None
    _lib.oracle_fgs.argtypes = [C.c_int, pd, pd, C.c_int, pd]
    _lib.oracle_sstep_step.restype = C.c_int
    _lib.oracle_sstep_step.argtypes = [i64, pi, pi, pd, pd, pd, pd, C.c_int, C.c_int, d, d, C.c_int, C.c_int,
                                       C.c_int, pd, pd, pd, pd, pd, pd, pd, pd, pd, pd]
    _lib.oracle_sstep_solve.restype = C.c_int
    _lib.oracle_sstep_solve.argtypes = [i64, pi, pi, pd, pd, pd, C.c_int, C.c_int, d, d, d, C.c_int, C.c_int,
                                        C.c_int, C.c_int, C.POINTER(C.c_int), pd, pd, pd, pd, pd, C.c_int]
    _lib.oracle_lanczos.restype = C.c_int
    _lib.oracle_lanczos.argtypes = [i64, pi, pi, pd, C.c_int, pd, C.c_int, pd, pd]
    _lib.oracle_prolongation_trilinear.restype = i64
    _lib.oracle_prolongation_trilinear.argtypes = [i32, i32, i32, pi, pi, pd]
    _lib.oracle_gs.restype = C.c_int
    _lib.oracle_gs.argtypes = [i64, pi, pi, pd, pd, C.c_int, pd]
    _lib.oracle_grad_csr.restype = None
    _lib.oracle_grad_csr.argtypes = [i64, pi, pi, pd, pd, pd]
    _lib.oracle_grad_faces.restype = None
    _lib.oracle_grad_faces.argtypes = [i32, i32, i32, pd, pd, pd, pd, pd]
    return _lib


def _pd(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _pi(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _csr(A):
    rp, ci, v = A
    return (np.ascontiguousarray(rp, dtype=np.int32), np.ascontiguousarray(ci, dtype=np.int32), _f64(v))


# ---------------------------------------------------------------------------

def dot(u, v) -> float:
    u, v = _f64(u), _f64(v)
    return _load().oracle_dot(u.size, _pd(u), _pd(v))


def csr_valid(n, A) -> bool:
    rp, ci, _ = _csr(A)
    return _load().oracle_csr_validate(n, _pi(rp), _pi(ci)) == 0


def spmv(A, x):
    rp, ci, v = _csr(A)
    x = _f64(x)
    y = np.empty(rp.size - 1)
    _load().oracle_spmv(rp.size - 1, _pi(rp), _pi(ci), _pd(v), _pd(x), _pd(y))
    return y


def assemble_stencil7(nx, ny, nz, kx=None, ky=None, kz=None):
    """CSR of the 7-point (face-coefficient) operator, assembled by the oracle."""
    lib = _load()
    n = nx * ny * nz
    nnz = lib.oracle_stencil7_nnz(nx, ny, nz)
    rp = np.empty(n + 1, np.int32)
    ci = np.empty(nnz, np.int32)
    v = np.empty(nnz)
    kx, ky, kz = _f64(kx), _f64(ky), _f64(kz)
    got = lib.oracle_assemble_stencil7(nx, ny, nz, _pd(kx), _pd(ky), _pd(kz), _pi(rp), _pi(ci), _pd(v))
    assert got == nnz
    return rp, ci, v


def assemble_stencil27(nx, ny, nz):
    """CSR of the 27-point operator (diagonal 26, -1 on the 26 neighbours of
    the 3 x 3 x 3 box inside the grid), assembled by the oracle."""
    lib = _load()
    n = nx * ny * nz
    nnz = lib.oracle_stencil27_nnz(nx, ny, nz)
    rp = np.empty(n + 1, np.int32)
    ci = np.empty(nnz, np.int32)
    v = np.empty(nnz)
    got = lib.oracle_assemble_stencil27(nx, ny, nz, _pi(rp), _pi(ci), _pd(v))
    assert got == nnz
    return rp, ci, v


def jacobi(A, precond=1):
    rp, ci, v = _csr(A)
    n = rp.size - 1
    invd = np.empty(n)
    dv = np.empty(n)
    st = _load().oracle_jacobi(n, _pi(rp), _pi(ci), _pd(v), precond, _pd(invd), _pd(dv))
    if st:
        raise ValueError("non-positive or missing diagonal")
    return invd, dv


def chebyshev_basis(A, invd, p0, s, lmin, lmax):
    """Columns p_0..p_{s-1} of the Chebyshev basis and A p_j (each n x s,
    returned as arrays of shape (s, n))."""
    rp, ci, v = _csr(A)
    n = rp.size - 1
    P = np.zeros((s, n))
    AP = np.zeros((s, n))
    P[0] = p0
    theta = 2.0 / (lmax - lmin)
    sigma = (lmax + lmin) / 2.0
    _load().oracle_chebyshev_basis(n, _pi(rp), _pi(ci), _pd(v), _pd(_f64(invd)), s, theta, sigma, _pd(P), _pd(AP))
    return P, AP


def gram(P, AP, r):
    s, n = P.shape
    G = np.empty((s, s))
    c = np.empty(s)
    _load().oracle_gram(n, s, _pd(_f64(P)), _pd(_f64(AP)), _pd(_f64(r)), _pd(G), _pd(c))
    return G, c


def column_scale(Graw, c):
    s = Graw.shape[0]
    G = np.empty((s, s))
    ct = np.empty(s)
    d = np.empty(s)
    st = _load().oracle_column_scale(s, _pd(_f64(Graw)), _pd(_f64(c)), _pd(G), _pd(ct), _pd(d))
    return st, G, ct, d


def fgs(G, ctil, nu):
    s = G.shape[0]
    a = np.empty(s)
    _load().oracle_fgs(s, _pd(_f64(G)), _pd(_f64(ctil)), nu, _pd(a))
    return a


BASIS = {"chebyshev": 0, "monomial": 1}


def step(A, b, xk, s, nu, lmin, lmax, precond=1, p0_mode=0, want_basis=False, basis="chebyshev"):
    """One outer iteration from ``xk``.  Returns a dict with ``status``,
    ``x`` (x_{k+1}), ``atil``, ``G``, ``ctil``, ``Graw``, ``d``, ``rnorm``,
    ``delta`` (Gram-solve residual, Sec. 7), ``lnorm`` (||L||_F, Sec. 4) and,
    with ``want_basis``, ``P`` / ``AP`` of shape (s, n).  ``basis`` is
    ``"chebyshev"`` (Sec. 2) or ``"monomial"`` (p_{j+1} = M^{-1} A p_j, the
    comparison of Sec. 4)."""
    rp, ci, v = _csr(A)
    n = rp.size - 1
    b, xk = _f64(b), _f64(xk)
    xn = np.empty(n)
    out = dict(atil=np.zeros(s), G=np.zeros((s, s)), ctil=np.zeros(s), Graw=np.zeros((s, s)), d=np.zeros(s),
               rnorm=np.zeros(1), delta=np.zeros(1), lnorm=np.zeros(1))
    P = np.zeros((s, n)) if want_basis else None
    AP = np.zeros((s, n)) if want_basis else None
    st = _load().oracle_sstep_step(n, _pi(rp), _pi(ci), _pd(v), _pd(b), _pd(xk), _pd(xn), s, nu, lmin, lmax,
                                   precond, p0_mode, BASIS[basis], _pd(out["atil"]), _pd(out["G"]), _pd(out["ctil"]),
                                   _pd(out["Graw"]), _pd(out["d"]), _pd(out["rnorm"]), _pd(out["delta"]),
                                   _pd(out["lnorm"]), _pd(P), _pd(AP))
    out.update(status=st, x=xn, rnorm=float(out["rnorm"][0]), delta=float(out["delta"][0]),
               lnorm=float(out["lnorm"][0]))
    if want_basis:
        out.update(P=P, AP=AP)
    return out


def solve(A, b, x0, s, nu, lmin, lmax, tol, max_outer=10000, precond=1, p0_mode=0, hist_cap=0, basis="chebyshev"):
    """Full solve; returns a dict with ``status``, ``x``, ``iters``,
    ``relres``, ``res0`` and the histories when ``hist_cap > 0``."""
    rp, ci, v = _csr(A)
    n = rp.size - 1
    b = _f64(b)
    x = np.array(x0, dtype=np.float64, copy=True) if x0 is not None else np.zeros(n)
    it = C.c_int(0)
    rel = np.zeros(1)
    r0 = np.zeros(1)
    hr = np.zeros(hist_cap) if hist_cap else None
    hd = np.zeros(hist_cap) if hist_cap else None
    hl = np.zeros(hist_cap) if hist_cap else None
    st = _load().oracle_sstep_solve(n, _pi(rp), _pi(ci), _pd(v), _pd(b), _pd(x), s, nu, lmin, lmax, tol, max_outer,
                                    precond, p0_mode, BASIS[basis], C.byref(it), _pd(rel), _pd(r0), _pd(hr), _pd(hd), _pd(hl),
                                    hist_cap)
    out = dict(status=st, x=x, iters=it.value, relres=float(rel[0]), res0=float(r0[0]))
    if hist_cap:
        k = min(it.value, hist_cap)
        out.update(hist_relres=hr[:min(it.value + 1, hist_cap)], hist_delta=hd[:k], hist_lnorm=hl[:k])
    return out


def lanczos(A, u, steps, precond=1):
    """Lanczos on M^{-1}A in the M-inner product (Sec. 8 setup) from start
    vector ``u``: returns dict ``alpha``, ``beta`` (length m <= steps, beta[i]
    below row i), the Ritz values ``ritz`` (eigenvalues of the m x m
    tridiagonal T_m, ascending; LAPACK's symmetric tridiagonal solver as the
    step) and ``m``."""
    rp, ci, v = _csr(A)
    n = rp.size - 1
    al = np.zeros(steps)
    be = np.zeros(steps)
    m = _load().oracle_lanczos(n, _pi(rp), _pi(ci), _pd(v), precond, _pd(_f64(u)), steps, _pd(al), _pd(be))
    al, be = al[:m], be[:m]
    if m == 0:
        ritz = np.zeros(0)
    else:
        import scipy.linalg
        ritz = scipy.linalg.eigvalsh_tridiagonal(al, be[:m - 1]) if m > 1 else al.copy()
    return dict(alpha=al, beta=be, ritz=np.sort(ritz), m=m)


def lanczos_bounds(ritz, margin=0.1):
    """Chebyshev bounds from the extreme Ritz values with a relative safety
    margin (Sec. 8: 10%): [(1 - margin) theta_min, (1 + margin) theta_max]."""
    return (1.0 - margin) * float(ritz[0]), (1.0 + margin) * float(ritz[-1])


def prolongation(ncx, ncy, ncz):
    """CSR (n_f x n_c) of the trilinear prolongation from the coarse grid to
    the (2 nc + 1)-point fine grid per axis (Sec. 6 two-level hierarchy)."""
    nf = (2 * ncx + 1) * (2 * ncy + 1) * (2 * ncz + 1)
    nc = ncx * ncy * ncz
    rp = np.empty(nf + 1, np.int32)
    ci = np.empty(27 * nc, np.int32)
    v = np.empty(27 * nc)
    nnz = _load().oracle_prolongation_trilinear(ncx, ncy, ncz, _pi(rp), _pi(ci), _pd(v))
    return rp, ci[:nnz].copy(), v[:nnz].copy()


def galerkin(Af, P, nc):
    """A_c = P^T A_f P formed explicitly (SciPy's sparse products as the
    step), returned as CSR with sorted columns."""
    import scipy.sparse as sp
    rp, ci, v = _csr(Af)
    nf = rp.size - 1
    A = sp.csr_matrix((v, ci, rp), shape=(nf, nf))
    Pm = sp.csr_matrix((P[2], P[1], P[0]), shape=(nf, nc))
    Ac = (Pm.T @ (A @ Pm)).tocsr()
    Ac.sort_indices()
    return Ac.indptr.astype(np.int32), Ac.indices.astype(np.int32), Ac.data.astype(np.float64)


def gs(A, f, nu):
    """nu forward Gauss-Seidel sweeps on A u = f from u = 0 (natural order)."""
    rp, ci, v = _csr(A)
    n = rp.size - 1
    u = np.empty(n)
    st = _load().oracle_gs(n, _pi(rp), _pi(ci), _pd(v), _pd(_f64(f)), nu, _pd(u))
    if st:
        raise ValueError("non-positive or missing diagonal")
    return u


def coarse_fgs(nc_dims, kx, ky, kz, f, nu):
    """The coarse-grid solve of the two-level hierarchy: A_f the 7-point
    face-coefficient operator on the fine grid (2 nc + 1 per axis), A_c =
    P^T A_f P formed, then nu FGS sweeps on A_c u = f from zero.  Returns
    (u, A_c)."""
    ncx, ncy, ncz = nc_dims
    Af = assemble_stencil7(2 * ncx + 1, 2 * ncy + 1, 2 * ncz + 1, kx, ky, kz)
    Ac = galerkin(Af, prolongation(ncx, ncy, ncz), ncx * ncy * ncz)
    return gs(Ac, f, nu), Ac


def gram_condition(G) -> float:
    """2-norm condition number of a symmetric positive definite Gram matrix
    (Sec. 4 and the measured values of Sec. 8), from its extreme eigenvalues
    (LAPACK's symmetric eigensolver as the step); inf when G is singular or
    indefinite in working precision."""
    w = np.linalg.eigvalsh(np.asarray(G, dtype=np.float64))
    return float(w[-1] / w[0]) if w[0] > 0 else float("inf")


def grad_csr(A, lam, x):
    rp, ci, _ = _csr(A)
    n = rp.size - 1
    dv = np.empty(ci.size)
    _load().oracle_grad_csr(n, _pi(rp), _pi(ci), _pd(_f64(lam)), _pd(_f64(x)), _pd(dv))
    return dv


def grad_faces(nx, ny, nz, lam, x):
    dkx = np.empty(nz * ny * (nx + 1))
    dky = np.empty(nz * (ny + 1) * nx)
    dkz = np.empty((nz + 1) * ny * nx)
    _load().oracle_grad_faces(nx, ny, nz, _pd(_f64(lam)), _pd(_f64(x)), _pd(dkx), _pd(dky), _pd(dkz))
    return dkx, dky, dkz


def problem_csr(pr):
    """CSR of a generated problem as the oracle sees it: 2D problems come as
    CSR from the generator; 3D stencil problems are assembled by the oracle
    itself from the grid and face coefficients."""
    if len(pr.dims) == 2:
        return _csr(pr.csr())
    nx, ny, nz = pr.dims
    if getattr(pr, "stencil", 7) == 27:
        return assemble_stencil27(nx, ny, nz)
    return assemble_stencil7(nx, ny, nz, pr.kx, pr.ky, pr.kz)
