"""Seeded synthetic problems (no solver arithmetic lives here).

Conventions
-----------
* Unknowns of an ``nx x ny (x nz)`` interior grid are numbered lexicographically
  with x fastest: ``idx = i + nx * (j + ny * k)``.
* Homogeneous Dirichlet boundary: neighbours outside the grid are dropped.
* Face coefficients of the variable-coefficient 7-point operator are stored
  x fastest as ``kx[k, j, i]`` of shape ``(nz, ny, nx + 1)`` (face between
  cells ``i-1`` and ``i``; ``i = 0`` and ``i = nx`` are boundary faces),
  ``ky`` of shape ``(nz, ny + 1, nx)`` and ``kz`` of shape ``(nz + 1, ny, nx)``.
  The operator is ``(A u)_p = sum over the 6 faces f of p of k_f (u_p - u_q)``
  with ``u_q = 0`` outside the grid, i.e. ``A_pp = sum_f k_f`` and
  ``A_pq = -k_f``.  With every ``k_f = 1`` it is the standard 7-point Poisson
  matrix (diagonal 6, off-diagonal -1).
* The workloads follow the paper's experiments (Sec. 8: 3D Poisson on the unit
  cube, Dirichlet boundary) at the sizes of the synthetic configurations
  listed in ``CONFIGS``.

Random streams use NumPy's PCG64 ``default_rng(seed)`` with a fixed draw order:
grid sizes, then ``kx``, ``ky``, ``kz`` (C order), then right-hand sides.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "rng", "uniform", "poisson2d_csr", "poisson3d_csr", "faces3d_csr",
    "face_coefficients", "jacobi_poisson_bounds", "gershgorin_jacobi_bounds",
    "poisson27_csr", "jacobi_poisson27_bounds",
    "Problem", "config1", "config2", "config3_sweep", "config4", "config5", "paper27", "TwoLevel", "two_level",
    "small_poisson3d", "small_faces3d", "small_poisson27", "CONFIGS",
]


def rng(seed: int) -> np.random.Generator:
    """PCG64 generator for ``seed`` (NumPy ``default_rng``)."""
    return np.random.default_rng(seed)


def uniform(r: np.random.Generator, n: int) -> np.ndarray:
    """``n`` iid draws from U[-1, 1] as float64."""
    return r.uniform(-1.0, 1.0, size=n)


# ---------------------------------------------------------------------------
# operators (CSR, int32 indices, float64 values, sorted columns)
# ---------------------------------------------------------------------------

def _csr_from_bands(n: int, cols: np.ndarray, vals: np.ndarray, mask: np.ndarray):
    """Pack an ``(n, w)`` band description (already in ascending column order
    within each row) into CSR arrays, keeping entries where ``mask`` is true."""
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32 indices")
    col_idx = cols[mask].astype(np.int32)
    val = vals[mask].astype(np.float64)
    return row_ptr.astype(np.int32), col_idx, val


def poisson2d_csr(nx: int, ny: int):
    """5-point Dirichlet Poisson matrix on an ``nx x ny`` interior grid
    (diagonal 4, off-diagonal -1).  Returns ``(row_ptr, col_idx, val)``."""
    n = nx * ny
    p = np.arange(n, dtype=np.int64)
    i = p % nx
    j = p // nx
    offs = [(-nx, j > 0), (-1, i > 0), (0, np.ones(n, bool)), (1, i < nx - 1), (nx, j < ny - 1)]
    cols = np.stack([p + o for o, _ in offs], axis=1)
    mask = np.stack([m for _, m in offs], axis=1)
    vals = np.where(cols == p[:, None], 4.0, -1.0)
    return _csr_from_bands(n, cols, vals, mask)


def poisson3d_csr(nx: int, ny: int, nz: int):
    """7-point Dirichlet Poisson matrix (diagonal 6, off-diagonal -1)."""
    return faces3d_csr(nx, ny, nz, None, None, None)


def faces3d_csr(nx: int, ny: int, nz: int, kx, ky, kz):
    """7-point operator from face coefficients (module docstring); ``None``
    coefficients mean the constant Poisson operator.  The diagonal is summed in
    the fixed face order west, east, south, north, bottom, top."""
    n = nx * ny * nz
    p = np.arange(n, dtype=np.int64)
    i = p % nx
    j = (p // nx) % ny
    k = p // (nx * ny)
    nxy = nx * ny
    if kx is None:
        one = np.ones(n)
        fw = fe = fs = fn = fb = ft = one
        diag = np.full(n, 6.0)
    else:
        kx = np.asarray(kx, dtype=np.float64).reshape(nz, ny, nx + 1)
        ky = np.asarray(ky, dtype=np.float64).reshape(nz, ny + 1, nx)
        kz = np.asarray(kz, dtype=np.float64).reshape(nz + 1, ny, nx)
        fw = kx[k, j, i]
        fe = kx[k, j, i + 1]
        fs = ky[k, j, i]
        fn = ky[k, j + 1, i]
        fb = kz[k, j, i]
        ft = kz[k + 1, j, i]
        diag = ((((fw + fe) + fs) + fn) + fb) + ft
    cols = np.stack([p - nxy, p - nx, p - 1, p, p + 1, p + nx, p + nxy], axis=1)
    vals = np.stack([-fb, -fs, -fw, diag, -fe, -fn, -ft], axis=1)
    mask = np.stack([k > 0, j > 0, i > 0, np.ones(n, bool), i < nx - 1, j < ny - 1, k < nz - 1], axis=1)
    return _csr_from_bands(n, cols, vals, mask)


def poisson27_csr(nx: int, ny: int, nz: int):
    """27-point Dirichlet operator: diagonal 26 and -1 for each of the 26
    neighbours of the 3 x 3 x 3 box inside the grid (columns ascending)."""
    n = nx * ny * nz
    p = np.arange(n, dtype=np.int64)
    i = p % nx
    j = (p // nx) % ny
    k = p // (nx * ny)
    cols, vals, masks = [], [], []
    for dk in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                cols.append(p + di + nx * (dj + ny * dk))
                vals.append(np.full(n, 26.0 if (di, dj, dk) == (0, 0, 0) else -1.0))
                masks.append((i + di >= 0) & (i + di < nx) & (j + dj >= 0) & (j + dj < ny)
                             & (k + dk >= 0) & (k + dk < nz))
    return _csr_from_bands(n, np.stack(cols, axis=1), np.stack(vals, axis=1), np.stack(masks, axis=1))


def face_coefficients(r: np.random.Generator, nx: int, ny: int, nz: int, sigma: float):
    """Log-normal face coefficients ``k_f = exp(sigma * Z)``, ``Z ~ N(0, 1)``,
    boundary faces included; drawn in the order kx, ky, kz (C order)."""
    kx = np.exp(sigma * r.standard_normal((nz, ny, nx + 1)))
    ky = np.exp(sigma * r.standard_normal((nz, ny + 1, nx)))
    kz = np.exp(sigma * r.standard_normal((nz + 1, ny, nx)))
    return kx.ravel(), ky.ravel(), kz.ravel()


# ---------------------------------------------------------------------------
# Chebyshev bounds: they must contain the spectrum of M^{-1} A (Sec. 2, Def.)
# ---------------------------------------------------------------------------

def jacobi_poisson_bounds(*dims: int):
    """Exact extreme eigenvalues of ``D^{-1} A`` for the constant-coefficient
    Dirichlet Poisson matrix on a ``d``-dimensional grid (``d = len(dims)``).
    The eigenvalues of ``A`` are ``2d - 2 sum_a cos(m_a pi/(N_a+1))`` and the
    diagonal is ``2d``, so the Jacobi-preconditioned spectrum is
    ``1 -/+ (1/d) sum_a cos(pi/(N_a+1))``."""
    d = len(dims)
    c = sum(math.cos(math.pi / (na + 1)) for na in dims) / d
    return 1.0 - c, 1.0 + c


def jacobi_poisson27_bounds(nx: int, ny: int, nz: int):
    """Exact extreme eigenvalues of ``D^{-1} A`` for the 27-point operator
    ``A = 27 I - T_x (x) T_y (x) T_z`` (``T`` = tridiag(1, 1, 1), eigenvalues
    ``1 + 2 cos(m pi/(N+1))``), diagonal 26: ``(27 - prod_a f_a) / 26``.  The
    product is multilinear in the three factors, so its extremes over the
    factor ranges ``[1 - 2c_a, 1 + 2c_a]``, ``c_a = cos(pi/(N_a+1))``, sit at
    the 8 corners."""
    c = [math.cos(math.pi / (na + 1)) for na in (nx, ny, nz)]
    prods = [a * b * d for a in (1 - 2 * c[0], 1 + 2 * c[0]) for b in (1 - 2 * c[1], 1 + 2 * c[1])
             for d in (1 - 2 * c[2], 1 + 2 * c[2])]
    return (27.0 - max(prods)) / 26.0, (27.0 - min(prods)) / 26.0


def gershgorin_jacobi_bounds():
    """Gershgorin interval of ``D^{-1} A`` for the face-coefficient operator:
    every disc has centre 1 and radius <= 1, hence ``[0, 2]``."""
    return 0.0, 2.0


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    """One linear system (or a family sharing an operator) plus solver settings.

    ``kind`` is ``"csr"`` or ``"stencil"``.  For ``"stencil"`` the grid and the
    optional face arrays define the operator; ``csr()`` assembles the same
    operator as a matrix.  ``xstar`` is the manufactured solution (``b = A x*``
    is formed by whoever consumes the problem); ``rhs`` holds explicit
    right-hand sides when there is no manufactured solution.
    """
    name: str
    kind: str
    dims: tuple
    s: int
    nu: int
    lmin: float
    lmax: float
    tol: float = 1e-8
    kx: np.ndarray | None = None
    ky: np.ndarray | None = None
    kz: np.ndarray | None = None
    xstar: np.ndarray | None = None
    rhs: list = field(default_factory=list)
    xtarget: np.ndarray | None = None
    stencil: int = 7
    _csr: tuple | None = None

    @property
    def n(self) -> int:
        return int(np.prod(self.dims))

    def csr(self):
        if self._csr is None:
            if len(self.dims) == 2:
                self._csr = poisson2d_csr(*self.dims)
            elif self.stencil == 27:
                self._csr = poisson27_csr(*self.dims)
            else:
                self._csr = faces3d_csr(*self.dims, self.kx, self.ky, self.kz)
        return self._csr


def config1(seed: int = 0) -> Problem:
    """2D 5-point Poisson, 64 x 64 interior (n = 4096), CSR, s = 8, nu = 20,
    exact Jacobi bounds, x* ~ U[-1, 1]."""
    r = rng(seed)
    lmin, lmax = jacobi_poisson_bounds(64, 64)
    return Problem("c1_poisson2d_64", "csr", (64, 64), 8, 20, lmin, lmax, xstar=uniform(r, 64 * 64))


def config2(seed: int = 0, N: int = 224, kind: str = "stencil", s: int = 16, nu: int = 25) -> Problem:
    """3D 7-point Poisson, ``N^3`` interior (224^3 = 11,239,424 unknowns),
    matrix-free stencil or CSR, s = 16, nu = 25, exact Jacobi bounds."""
    r = rng(seed)
    lmin, lmax = jacobi_poisson_bounds(N, N, N)
    return Problem(f"c2_poisson3d_{N}_{kind}", kind, (N, N, N), s, nu, lmin, lmax,
                   xstar=uniform(r, N ** 3))


def config3_sweep():
    """(s, nu) pairs of the mixed-precision sweep on the 224^3 problem."""
    return [(s, nu) for s in (8, 16, 24, 32) for nu in (20, 30)]


def config4(seed: int = 0, nsys: int = 64, nrhs: int = 8, nmin: int = 32, nmax: int = 96,
            sigma: float = 1.0, s: int = 16, nu: int = 25):
    """Batched variable-coefficient diffusion: ``nsys`` cubic grids with
    ``N_i ~ U{nmin..nmax}``, log-normal faces (sigma), ``nrhs`` right-hand sides
    U[-1, 1] each, Gershgorin bounds [0, 2]."""
    r = rng(seed)
    sizes = r.integers(nmin, nmax + 1, size=nsys)
    lmin, lmax = gershgorin_jacobi_bounds()
    probs = []
    for q, N in enumerate(sizes):
        N = int(N)
        kx, ky, kz = face_coefficients(r, N, N, N, sigma)
        probs.append(Problem(f"c4_sys{q}_{N}", "stencil", (N, N, N), s, nu, lmin, lmax,
                             kx=kx, ky=ky, kz=kz))
    for pr in probs:
        pr.rhs = [uniform(r, pr.n) for _ in range(nrhs)]
    return probs


def config5(seed: int = 0, N: int = 128, sigma: float = 0.5, s: int = 16, nu: int = 25) -> Problem:
    """Differentiable diffusion solve: ``N^3`` grid, log-normal faces (sigma),
    b and x_target ~ U[-1, 1], Gershgorin bounds [0, 2]."""
    r = rng(seed)
    kx, ky, kz = face_coefficients(r, N, N, N, sigma)
    lmin, lmax = gershgorin_jacobi_bounds()
    pr = Problem(f"c5_diffusion_{N}", "stencil", (N, N, N), s, nu, lmin, lmax, kx=kx, ky=ky, kz=kz)
    pr.rhs = [uniform(r, pr.n)]
    pr.xtarget = uniform(r, pr.n)
    return pr


def paper27(seed: int = 0, N: int = 230, s: int = 20, nu: int = 30) -> Problem:
    """The paper's own workload (Sec. 8): 3D Poisson on the unit cube with a
    27-point stencil, Dirichlet boundary, 230^3 = 12,167,000 unknowns (about
    12.2M per GPU), s in {10, 20}, nu in {6, 15, 30}; x* ~ U[-1, 1], b = A x*.
    The bounds given here are the exact Jacobi bounds; the paper's runs take
    them from 10 Lanczos steps with a 10% margin."""
    r = rng(seed)
    lmin, lmax = jacobi_poisson27_bounds(N, N, N)
    return Problem(f"paper27_poisson3d_{N}", "stencil", (N, N, N), s, nu, lmin, lmax, xstar=uniform(r, N ** 3),
                   stencil=27)


def small_poisson27(nx: int, ny: int, nz: int, seed: int = 0, s: int = 8, nu: int = 25) -> Problem:
    """Small 27-point Poisson problem (exact Jacobi bounds), x* ~ U[-1, 1]."""
    r = rng(seed)
    lmin, lmax = jacobi_poisson27_bounds(nx, ny, nz)
    return Problem(f"poisson27_{nx}x{ny}x{nz}", "stencil", (nx, ny, nz), s, nu, lmin, lmax,
                   xstar=uniform(r, nx * ny * nz), stencil=27)


@dataclass
class TwoLevel:
    """A synthetic two-level hierarchy (Sec. 6; Sec. 8 streaming coarse solve):
    coarse grid ``nc`` points per axis, fine grid ``2 nc + 1``, log-normal face
    coefficients of the fine 7-point operator, a coarse right-hand side, nu
    coarse FGS sweeps."""
    nc: tuple
    kx: np.ndarray
    ky: np.ndarray
    kz: np.ndarray
    f: np.ndarray
    nu: int = 20

    @property
    def nf(self) -> tuple:
        return tuple(2 * c + 1 for c in self.nc)

    @property
    def n_coarse(self) -> int:
        return int(np.prod(self.nc))


def two_level(seed: int = 0, nc=(17, 17, 17), sigma: float = 1.0, nu: int = 20) -> TwoLevel:
    """Coarse 17^3 = 4913 unknowns (about the paper's n_c = 5000), fine
    35^3; faces k_f = exp(sigma Z) drawn kx, ky, kz; f ~ U[-1, 1]."""
    r = rng(seed)
    fx, fy, fz = (2 * c + 1 for c in nc)
    kx, ky, kz = face_coefficients(r, fx, fy, fz, sigma)
    return TwoLevel(tuple(nc), kx, ky, kz, uniform(r, int(np.prod(nc))), nu)


def small_poisson3d(nx: int, ny: int, nz: int, seed: int = 0, s: int = 8, nu: int = 25) -> Problem:
    """Small constant-coefficient 3D Poisson problem (exact Jacobi bounds)."""
    r = rng(seed)
    lmin, lmax = jacobi_poisson_bounds(nx, ny, nz)
    return Problem(f"poisson3d_{nx}x{ny}x{nz}", "stencil", (nx, ny, nz), s, nu, lmin, lmax,
                   xstar=uniform(r, nx * ny * nz))


def small_faces3d(nx: int, ny: int, nz: int, seed: int = 0, sigma: float = 1.0, s: int = 8,
                  nu: int = 25) -> Problem:
    """Small variable-coefficient problem (Gershgorin bounds), x* ~ U[-1, 1]."""
    r = rng(seed)
    kx, ky, kz = face_coefficients(r, nx, ny, nz, sigma)
    lmin, lmax = gershgorin_jacobi_bounds()
    return Problem(f"faces3d_{nx}x{ny}x{nz}", "stencil", (nx, ny, nz), s, nu, lmin, lmax,
                   kx=kx, ky=ky, kz=kz, xstar=uniform(r, nx * ny * nz))


CONFIGS = {
    "c1": config1,
    "c2": config2,
    "c4": config4,
    "c5": config5,
}
