"""Python front end of the s-step CG library: thin wrappers that marshal torch
tensors (device memory, streams) into the C ABI.  Every step of the method
runs in the HIP kernels behind the ABI."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _native as N


def require_gpu() -> None:
    """Raise unless a GPU and the built HIP library are both available."""
    N.load()
    if not torch.cuda.is_available():
        raise RuntimeError("no ROCm GPU is visible to torch")


def _check(status: int, ctx=None, stats=None):
    if status != N.SSTEP_OK:
        raise N.SStepError(status, N.last_error(ctx), stats)


def _host_or_device(a, dtype):
    """(pointer, ptr_space, keep-alive) for a numpy array or torch tensor."""
    if a is None:
        return None, 0, None
    if isinstance(a, torch.Tensor):
        t = a.detach().to(dtype=dtype).contiguous()
        return t.data_ptr(), (1 if t.is_cuda else 0), t
    arr = np.ascontiguousarray(a, dtype={torch.float64: np.float64, torch.int32: np.int32}[dtype])
    return arr.ctypes.data, 0, arr


@dataclass
class Operator:
    """A sparse SPD operator: CSR arrays or a 7-point stencil grid with
    optional face coefficients (layouts as in ``include/sstep.h``)."""
    kind: int
    n: int
    nnz: int = 0
    row_ptr: object = None
    col_idx: object = None
    val: object = None
    dims: tuple = ()
    kx: object = None
    ky: object = None
    kz: object = None
    _keep: list = field(default_factory=list, repr=False)

    @staticmethod
    def csr(row_ptr, col_idx, val) -> "Operator":
        n = len(row_ptr) - 1
        return Operator(N.OP_CSR, n, int(len(col_idx)), row_ptr, col_idx, val)

    @staticmethod
    def stencil(nx: int, ny: int, nz: int, kx=None, ky=None, kz=None) -> "Operator":
        return Operator(N.OP_STENCIL7, nx * ny * nz, dims=(nx, ny, nz), kx=kx, ky=ky, kz=kz)

    @staticmethod
    def stencil27(nx: int, ny: int, nz: int) -> "Operator":
        """The 27-point Poisson operator (diagonal 26, -1 on the box)."""
        return Operator(N.OP_STENCIL27, nx * ny * nz, dims=(nx, ny, nz))

    @property
    def grad_size(self) -> int:
        if self.kind == N.OP_CSR:
            return self.nnz
        if self.kind == N.OP_STENCIL27:
            return 0
        nx, ny, nz = self.dims
        return (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)

    def split_faces(self, flat):
        """Split a concatenated [kx | ky | kz] vector into its three parts."""
        nx, ny, nz = self.dims
        a = (nx + 1) * ny * nz
        b = a + nx * (ny + 1) * nz
        return flat[:a], flat[a:b], flat[b:]

    def to_c(self) -> N.Operator:
        op = N.Operator()
        op.kind = self.kind
        keep = []
        spaces = set()
        if self.kind == N.OP_CSR:
            op.n, op.nnz = self.n, self.nnz
            for name, dt in (("row_ptr", torch.int32), ("col_idx", torch.int32), ("val", torch.float64)):
                p, sp, k = _host_or_device(getattr(self, name), dt)
                setattr(op, name, p)
                keep.append(k)
                spaces.add(sp)
        else:
            op.nx, op.ny, op.nz = self.dims
            for name in ("kx", "ky", "kz"):
                p, sp, k = _host_or_device(getattr(self, name), torch.float64)
                setattr(op, name, p)
                keep.append(k)
                if k is not None:
                    spaces.add(sp)
        if len(spaces) > 1:
            raise ValueError("operator arrays must all be host or all be device memory")
        op.ptr_space = spaces.pop() if spaces else 0
        self._keep = keep
        return op


def _dev_ptr(t: torch.Tensor, n: int, name: str) -> int:
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    if t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} entries, need {n}")
    return t.data_ptr()


@dataclass
class SolveStats:
    outer_iters: int
    status: int
    rel_res: float
    res0: float
    hist_relres: np.ndarray | None = None
    hist_delta: np.ndarray | None = None
    hist_lnorm: np.ndarray | None = None


class Solver:
    """s-step CG solver bound to one operator (one library context)."""

    def __init__(self, op: Operator, s: int, nu: int, lmin: float, lmax: float, *, precision: str = "fp64",
                 precond: bool = True, p0_mode: int = 0, max_outer: int = 10000, graph_chunk: int = 4,
                 record_history: bool = False, autotune: bool = True, gram: str = "auto", basis: str = "chebyshev",
                 basis_steps: int = 0, stream=None):
        self._lib = N.load()
        self.op = op
        self.s, self.nu, self.lmin, self.lmax = s, nu, lmin, lmax
        self.precision = precision
        opt = N.Options()
        self._lib.sstep_default_options(C.byref(opt))
        opt.precision = {"fp64": N.FP64, "fp32ir": N.FP32_IR}[precision]
        opt.precond = 1 if precond else 0
        opt.p0_mode = p0_mode
        opt.max_outer = max_outer
        opt.graph_chunk = graph_chunk
        opt.record_history = 1 if record_history else 0
        opt.autotune = 1 if autotune else 0
        opt.gram = N.GRAM_KINDS[gram]
        opt.basis = {"chebyshev": 0, "monomial": 1}[basis]
        opt.basis_steps = basis_steps
        self._stream = stream
        opt.stream = self._stream_ptr()
        self.max_outer = max_outer
        self.record_history = record_history
        self.coeff_token = None
        cop = op.to_c()
        ctx = C.c_void_p()
        st = self._lib.sstep_setup(C.byref(ctx), C.byref(cop), s, nu, lmin, lmax, C.byref(opt))
        op._keep = []
        _check(st, None)
        self._ctx = ctx
        self.n = int(self._lib.sstep_n(ctx))
        self.grad_size = int(self._lib.sstep_grad_size(ctx))
        # True when the Gram kernel forms A p_j itself (AP not kept, s - 1 basis launches)
        self.gram_applies_operator = bool(self._lib.sstep_gram_mode(ctx) == N.GRAM_KINDS["apply"])
        # "stored", "apply" or "recurrence": how this context forms G = P^T A P
        self.gram_kind = {v: k for k, v in N.GRAM_KINDS.items()}[int(self._lib.sstep_gram_mode(ctx))]
        pairs = C.c_int32(0)
        #: kernel launches per basis and how many of them form two columns
        self.basis_launches = int(self._lib.sstep_basis_launches(ctx, C.byref(pairs)))
        self.basis_pairs = int(pairs.value)

    def _stream_ptr(self):
        if self._stream is not None:
            return self._stream.cuda_stream
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
        return None

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.sstep_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------
    def update_coefficients(self, op: Operator):
        cop = op.to_c()
        st = self._lib.sstep_update_coefficients(self._ctx, C.byref(cop))
        op._keep = []
        self.coeff_token = None  # the differentiable solve's marker of which coefficients are loaded
        _check(st, self._ctx)

    def apply(self, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
        y = torch.empty_like(x) if y is None else y
        _check(self._lib.sstep_apply(self._ctx, _dev_ptr(x, self.n, "x"), _dev_ptr(y, self.n, "y")), self._ctx)
        return y

    def _solve(self, fn, b, x, tol, raise_on_error, hist):
        if x is None:
            x = torch.zeros_like(b)
        stats = N.Stats()
        cap = (self.max_outer + 1) if (hist and self.record_history) else 0
        hr = np.zeros(max(cap, 1))
        hd = np.zeros(max(cap, 1))
        hl = np.zeros(max(cap, 1))
        if cap:
            stats.hist_relres = hr.ctypes.data
            stats.hist_delta = hd.ctypes.data
            stats.hist_lnorm = hl.ctypes.data
            stats.hist_cap = cap
        st = fn(self._ctx, _dev_ptr(b, self.n, "b"), _dev_ptr(x, self.n, "x"), tol, C.byref(stats))
        out = SolveStats(stats.outer_iters, stats.status, stats.rel_res, stats.res0)
        if cap:
            out.hist_relres = hr[:stats.outer_iters + 1].copy()
            out.hist_delta = hd[:stats.outer_iters].copy()
            out.hist_lnorm = hl[:stats.outer_iters].copy()
        if raise_on_error:
            _check(st, self._ctx, out)
        return x, out

    def solve(self, b: torch.Tensor, x: torch.Tensor | None = None, tol: float = 1e-8, *,
              raise_on_error: bool = True, history: bool = False):
        """Solve A x = b in place in ``x`` (zeros if None); returns (x, stats)."""
        return self._solve(self._lib.sstep_solve, b, x, tol, raise_on_error, history)

    def solve_adjoint(self, g: torch.Tensor, lam: torch.Tensor | None = None, tol: float = 1e-8, *,
                      raise_on_error: bool = True, history: bool = False):
        return self._solve(self._lib.sstep_solve_adjoint, g, lam, tol, raise_on_error, history)

    def grad_operator(self, lam: torch.Tensor, x: torch.Tensor, out: torch.Tensor | None = None,
                      accumulate: bool = False) -> torch.Tensor:
        if out is None:
            out = torch.zeros(self.grad_size, dtype=torch.float64, device=x.device)
        _check(self._lib.sstep_grad_operator(self._ctx, _dev_ptr(lam, self.n, "lam"), _dev_ptr(x, self.n, "x"),
                                             _dev_ptr(out, self.grad_size, "dA"), 1 if accumulate else 0),
               self._ctx)
        return out

    def step(self, b: torch.Tensor, x: torch.Tensor, want_basis: bool = False) -> dict:
        """One outer iteration in place on ``x`` (parity entry point)."""
        s = self.s
        atil = np.zeros(s)
        G = np.zeros((s, s))
        ct = np.zeros(s)
        rn = np.zeros(1)
        P = AP = None
        if want_basis:
            P = torch.empty((s, self.n), dtype=torch.float64, device=x.device)
            AP = torch.empty((s, self.n), dtype=torch.float64, device=x.device)
        st = self._lib.sstep_step(self._ctx, _dev_ptr(b, self.n, "b"), _dev_ptr(x, self.n, "x"),
                                  atil.ctypes.data, G.ctypes.data, ct.ctypes.data, rn.ctypes.data,
                                  P.data_ptr() if P is not None else None,
                                  AP.data_ptr() if AP is not None else None)
        _check(st, self._ctx)
        out = dict(atil=atil, G=G, ctil=ct, rnorm=float(rn[0]), x=x)
        if want_basis:
            out.update(P=P, AP=AP)
        return out

    def lanczos(self, u: torch.Tensor, steps: int = 10) -> dict:
        """Lanczos on M^{-1}A from ``u`` (device float64): ``alpha``, ``beta``,
        ``ritz`` (ascending) of the ``m`` completed steps."""
        al, be, rz = np.zeros(steps), np.zeros(steps), np.zeros(steps)
        m = C.c_int32(0)
        _check(self._lib.sstep_lanczos(self._ctx, _dev_ptr(u, self.n, "u"), steps, al.ctypes.data, be.ctypes.data,
                                       rz.ctypes.data, C.byref(m)), self._ctx)
        k = m.value
        return dict(alpha=al[:k], beta=be[:k], ritz=rz[:k], m=k)

    def set_bounds(self, lmin: float, lmax: float):
        _check(self._lib.sstep_set_bounds(self._ctx, lmin, lmax), self._ctx)
        self.lmin, self.lmax = lmin, lmax

    def lanczos_bounds(self, u: torch.Tensor, steps: int = 10, margin: float = 0.1):
        """Sets the Chebyshev bounds from ``steps`` Lanczos steps with a
        relative ``margin`` (Sec. 8: 10 steps, 10%); returns (lmin, lmax)."""
        lo, hi = C.c_double(0.0), C.c_double(0.0)
        _check(self._lib.sstep_lanczos_bounds(self._ctx, _dev_ptr(u, self.n, "u"), steps, margin, C.byref(lo),
                                              C.byref(hi)), self._ctx)
        self.lmin, self.lmax = lo.value, hi.value
        return lo.value, hi.value

    def last_iteration(self) -> dict:
        """``rnorm``, ``delta`` (Gram-solve residual) and ``lnorm`` (||L||_F)
        of the last outer iteration (after ``step`` or a solve)."""
        v = np.zeros(3)
        _check(self._lib.sstep_last_iteration(self._ctx, v[0:].ctypes.data, v[1:].ctypes.data, v[2:].ctypes.data),
               self._ctx)
        return dict(rnorm=float(v[0]), delta=float(v[1]), lnorm=float(v[2]))

    def kernel_times(self, b: torch.Tensor, x_scratch: torch.Tensor, reps: int = 5) -> dict:
        """Average ms per launch of each kernel class (HIP events)."""
        ms = np.zeros(len(N.KT_NAMES))
        _check(self._lib.sstep_kernel_times(self._ctx, _dev_ptr(b, self.n, "b"), _dev_ptr(x_scratch, self.n, "x"),
                                            reps, ms.ctypes.data), self._ctx)
        return dict(zip(N.KT_NAMES, ms.tolist()))


class BatchedSolver:
    """Many stencil systems x ``nrhs`` right-hand sides, advanced together: one
    launch per step of the outer iteration covers every (system, rhs) pair."""

    def __init__(self, ops: list, nrhs: int, s: int, nu: int, lmin, lmax, *, precision: str = "fp64",
                 precond: bool = True, p0_mode: int = 0, max_outer: int = 10000, graph_chunk: int = 4,
                 autotune: bool = True, gram: str = "auto", basis_steps: int = 0, stream=None):
        self._lib = N.load()
        self.ops = list(ops)
        self.nsys = len(self.ops)
        self.nrhs = nrhs
        self.s, self.nu = s, nu
        opt = N.Options()
        self._lib.sstep_default_options(C.byref(opt))
        opt.precision = {"fp64": N.FP64, "fp32ir": N.FP32_IR}[precision]
        opt.precond = 1 if precond else 0
        opt.p0_mode = p0_mode
        opt.max_outer = max_outer
        opt.graph_chunk = graph_chunk
        opt.autotune = 1 if autotune else 0
        opt.gram = N.GRAM_KINDS[gram]
        opt.basis_steps = basis_steps
        self._stream = stream
        opt.stream = stream.cuda_stream if stream is not None else (
            torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None)
        carr = (N.Operator * self.nsys)(*[op.to_c() for op in self.ops])
        lo = np.ascontiguousarray(lmin, dtype=np.float64)
        hi = np.ascontiguousarray(lmax, dtype=np.float64)
        if lo.size != self.nsys or hi.size != self.nsys:
            raise ValueError("one (lmin, lmax) pair per system")
        ctx = C.c_void_p()
        st = self._lib.sstep_setup_batched(C.byref(ctx), self.nsys, carr, nrhs, s, nu, lo.ctypes.data,
                                           hi.ctypes.data, C.byref(opt))
        for op in self.ops:
            op._keep = []
        _check(st, None)
        self._ctx = ctx
        self.sizes = [op.n for op in self.ops]
        self.gram_kind = {v: k for k, v in N.GRAM_KINDS.items()}[int(self._lib.sstep_gram_mode(ctx))]
        rows, factor = C.c_int64(0), C.c_int32(0)
        _check(self._lib.sstep_batched_tiles(ctx, C.byref(rows), C.byref(factor)), ctx)
        #: the tile schedule: rows per chunk tile and persistent blocks per compute unit
        self.tiles = {"rows_per_tile": int(rows.value), "grid_factor": int(factor.value)}
        pairs = C.c_int32(0)
        #: kernel launches per basis and how many of them form two columns
        self.basis_launches = int(self._lib.sstep_basis_launches(ctx, C.byref(pairs)))
        self.basis_pairs = int(pairs.value)

    def bands(self):
        """(bands, tail_bands, tail_replays): blocks per right-hand side of the
        two-step basis's band table for the whole batch, of its short-range
        table for the end of a solve (0 when there is none), and the graph
        replays of the last solve that ran on the short ranges."""
        b, t, r = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        _check(self._lib.sstep_batched_bands(self._ctx, C.byref(b), C.byref(t), C.byref(r)), self._ctx)
        return int(b.value), int(t.value), int(r.value)

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.sstep_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def solve(self, b: list, x: list | None = None, tol: float = 1e-8, *, raise_on_error: bool = True):
        """``b[q]``, ``x[q]``: float64 CUDA tensors of n_q * nrhs entries
        (right-hand side r at offset r * n_q).  Returns (x, stats) with one
        SolveStats per pair, pair (q, r) at q * nrhs + r."""
        if len(b) != self.nsys:
            raise ValueError("one right-hand-side block per system")
        if x is None:
            x = [torch.zeros_like(bq) for bq in b]
        bp = (C.c_void_p * self.nsys)(*[_dev_ptr(bq, n * self.nrhs, "b") for bq, n in zip(b, self.sizes)])
        xp = (C.c_void_p * self.nsys)(*[_dev_ptr(xq, n * self.nrhs, "x") for xq, n in zip(x, self.sizes)])
        stats = (N.Stats * (self.nsys * self.nrhs))()
        st = self._lib.sstep_solve_batched(self._ctx, bp, xp, tol, stats)
        out = [SolveStats(v.outer_iters, v.status, v.rel_res, v.res0) for v in stats]
        if raise_on_error:
            _check(st, self._ctx)
        return x, out


class CoarseSolver:
    """Coarse-grid solve of a two-level hierarchy: ``nu`` forward Gauss-Seidel
    sweeps on A_c = P^T A_f P (trilinear P) from zero, with A_c never formed
    (``formed=False``) or formed on the device at setup (``formed=True``).
    ``fine_op`` is a 7-point stencil Operator on the (2 nc + 1)-point grid."""

    def __init__(self, fine_op: Operator, formed: bool = False, stream=None):
        self._lib = N.load()
        opt = N.Options()
        self._lib.sstep_default_options(C.byref(opt))
        opt.stream = stream.cuda_stream if stream is not None else (
            torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None)
        cop = fine_op.to_c()
        ctx = C.c_void_p()
        st = self._lib.sstep_coarse_setup(C.byref(ctx), C.byref(cop), 1 if formed else 0, C.byref(opt))
        fine_op._keep = []
        _check(st, None)
        self._ctx = ctx
        nc, nb = C.c_int64(0), C.c_int64(0)
        _check(self._lib.sstep_coarse_info(ctx, C.byref(nc), C.byref(nb)), ctx)
        self.n = nc.value
        self.workspace_bytes = nb.value
        self.formed = formed

    def fgs(self, f: torch.Tensor, nu: int, u: torch.Tensor | None = None) -> torch.Tensor:
        u = torch.empty_like(f) if u is None else u
        _check(self._lib.sstep_coarse_fgs(self._ctx, _dev_ptr(f, self.n, "f"), _dev_ptr(u, self.n, "u"), nu),
               self._ctx)
        return u

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.sstep_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
