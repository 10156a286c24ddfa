"""C-ABI checks that need no GPU: the library loads, exports every function
``include/sstep.h`` declares, and rejects invalid arguments before touching a
device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "sstep.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sstep_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def native():
    from paper_2512_09642_amd import _native
    return _native


def test_library_exports_every_declared_function(native):
    lib = native.load()
    names = header_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(native.EXPORTS)


def test_default_options_and_status_strings(native):
    lib = native.load()
    opt = native.Options()
    lib.sstep_default_options(C.byref(opt))
    assert (opt.precision, opt.precond, opt.p0_mode, opt.max_outer, opt.graph_chunk, opt.record_history,
            opt.autotune, opt.gram) == (0, 1, 0, 10000, 4, 0, 1, 0)
    assert lib.sstep_gram_mode(None) == -1
    assert lib.sstep_batched_bands(None, None, None, None) == 1  # SSTEP_E_ARG
    for code, name in native.STATUS_NAMES.items():
        assert lib.sstep_status_string(code).decode() == name


def _setup(native, op, s=4, nu=5, lmin=0.1, lmax=1.9):
    lib = native.load()
    ctx = C.c_void_p()
    st = lib.sstep_setup(C.byref(ctx), C.byref(op), s, nu, lmin, lmax, None)
    return st, ctx, lib.sstep_last_error(None).decode()


def _poisson(native, nx=4, ny=4, nz=4):
    op = native.Operator()
    op.kind = native.OP_STENCIL7
    op.nx, op.ny, op.nz = nx, ny, nz
    return op


@pytest.mark.parametrize("s,nu,lmin,lmax", [(0, 5, 0.1, 1.9), (33, 5, 0.1, 1.9), (4, 0, 0.1, 1.9),
                                             (4, 5, 1.9, 0.1), (4, 5, -1.0, 1.0), (4, 5, 0.1, float("inf")),
                                             (4, 5, float("nan"), 1.0)])
def test_setup_rejects_bad_parameters(native, s, nu, lmin, lmax):
    st, ctx, msg = _setup(native, _poisson(native), s, nu, lmin, lmax)
    assert st == 1 and not ctx.value and msg


def test_setup_rejects_bad_grids_and_faces(native):
    assert _setup(native, _poisson(native, 0, 4, 4))[0] == 1
    assert _setup(native, _poisson(native, 2048, 2048, 1024))[0] == 1  # n >= 2^31
    op = _poisson(native)
    k = np.ones(100)
    op.kx = k.ctypes.data  # one face array without the other two
    assert _setup(native, op)[0] == 1


def _csr(native, rp, ci, v):
    op = native.Operator()
    op.kind = native.OP_CSR
    op.ptr_space = 0
    op.n = len(rp) - 1
    op.nnz = len(ci)
    keep = [np.ascontiguousarray(rp, np.int32), np.ascontiguousarray(ci, np.int32), np.ascontiguousarray(v)]
    op.row_ptr, op.col_idx, op.val = (a.ctypes.data for a in keep)
    return op, keep


@pytest.mark.parametrize("case", ["col_range", "unsorted", "rowptr", "nnz"])
def test_setup_rejects_malformed_csr(native, case):
    rp = [0, 2, 4, 6]
    ci = [0, 1, 0, 1, 1, 2]
    v = [2.0, -1.0, -1.0, 2.0, -1.0, 2.0]
    if case == "col_range":
        ci = [0, 1, 0, 3, 1, 2]
    elif case == "unsorted":
        ci = [1, 0, 0, 1, 1, 2]
    elif case == "rowptr":
        rp = [0, 3, 2, 6]
    op, keep = _csr(native, rp, ci, v)
    if case == "nnz":
        op.nnz = 5
    st, ctx, msg = _setup(native, op)
    assert st == 1 and "CSR" in msg


def test_null_arguments(native):
    lib = native.load()
    ctx = C.c_void_p()
    assert lib.sstep_setup(C.byref(ctx), None, 4, 5, 0.1, 1.9, None) == 1
    assert lib.sstep_setup(None, None, 4, 5, 0.1, 1.9, None) == 1
    assert lib.sstep_solve(None, None, None, 1e-8, None) == 1
    assert lib.sstep_n(None) == 0
    lib.sstep_destroy(None)


def test_batched_entry_points_report_status(native):
    lib = native.load()
    ctx = C.c_void_p()
    st = lib.sstep_setup_batched(C.byref(ctx), 0, None, 1, 4, 5, None, None, None)
    assert st != 0


def test_setup_rejects_unavailable_gram_kinds(native):
    """The operator-applying Gram kernel needs a stencil operator, s <= 16 and
    columns under 4 GiB, the recurrence kind s <= 31, the moments kind s <= 31
    with the Chebyshev basis and p_0 = M^{-1} r (or no preconditioner); asking
    for them otherwise is unsupported, an unknown kind or option value is an
    argument error.  Checked before any device work."""
    lib = native.load()

    def setup(op, s, gram):
        opt = native.Options()
        lib.sstep_default_options(C.byref(opt))
        opt.gram = gram
        ctx = C.c_void_p()
        return lib.sstep_setup(C.byref(ctx), C.byref(op), s, 5, 0.1, 1.9, C.byref(opt)), ctx

    apply_op = native.GRAM_KINDS["apply"]
    st, ctx = setup(_poisson(native), 17, apply_op)
    assert st == 7 and not ctx.value
    rp = np.array([0, 1, 2]); ci = np.array([0, 1]); v = np.array([2.0, 2.0])
    op, keep = _csr(native, rp, ci, v)
    st, ctx = setup(op, 4, apply_op)
    assert st == 7 and not ctx.value
    st, ctx = setup(_poisson(native), 4, 9)
    assert st == 1 and not ctx.value
    # the recurrence kind needs the Gram of s + 1 <= 32 columns
    st, ctx = setup(_poisson(native), 32, native.GRAM_KINDS["recurrence"])
    assert st == 7 and not ctx.value
    # 820^3 doubles per column exceed the kernel's 32-bit byte offsets
    st, ctx = setup(_poisson(native, 820, 820, 820), 4, apply_op)
    assert st == 7 and not ctx.value
    # the moments kind: s <= 31, the Chebyshev basis, and c = P^T r in the M
    # inner product (p_0 = M^{-1} r, or no preconditioner)
    moments = native.GRAM_KINDS["moments"]
    st, ctx = setup(_poisson(native), 32, moments)
    assert st == 7 and not ctx.value

    def setup_opts(**kw):
        opt = native.Options()
        lib.sstep_default_options(C.byref(opt))
        opt.gram = moments
        for k, v in kw.items():
            setattr(opt, k, v)
        ctx = C.c_void_p()
        return lib.sstep_setup(C.byref(ctx), C.byref(_poisson(native)), 8, 5, 0.1, 1.9, C.byref(opt)), ctx

    st, ctx = setup_opts(p0_mode=1)
    assert st == 7 and not ctx.value
    st, ctx = setup_opts(basis=1)
    assert st == 7 and not ctx.value
    st, ctx = setup_opts(precision=native.FP32_IR)
    assert st == 7 and not ctx.value
    st, ctx = setup_opts(basis_steps=2)
    assert st == 1 and not ctx.value


def test_missing_library_fails_loudly(native, monkeypatch, tmp_path):
    """Without the built library the binding raises; there is no fallback."""
    monkeypatch.setattr(native, "_lib", None)
    monkeypatch.setattr(native, "LIB_PATH", str(tmp_path / "libsstep.so"))
    with pytest.raises(ImportError, match="no CPU fallback"):
        native.load()


def test_entry_point_build_runs(monkeypatch):
    """``__graft_entry__.build()`` reaches every step: the HIP build (stubbed
    here, it takes minutes), the oracle build and the package import."""
    import importlib
    import sys

    sys.path.insert(0, ROOT)
    entry = importlib.import_module("__graft_entry__")
    from paper_2512_09642_amd import build as hipbuild

    calls = []
    monkeypatch.setattr(hipbuild, "build", lambda *a, **k: calls.append("hip"))
    entry.build()
    assert calls == ["hip"]
    from oracle.build import LIB
    assert os.path.exists(LIB)
