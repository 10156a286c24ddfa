"""Drives the C ABI's host-side argument checks (no GPU needed: every call
here is rejected before the first HIP call).  Run in a subprocess by
tests/test_sanitizers.py against a library whose host code is built with
AddressSanitizer and UndefinedBehaviorSanitizer (path in argv[1])."""
import ctypes as C
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import paper_2512_09642_amd._native as N  # noqa: E402

N.LIB_PATH = sys.argv[1]
lib = N.load()


def csr_op(rp, ci, v):
    op = N.Operator()
    op.kind, op.ptr_space, op.n, op.nnz = N.OP_CSR, 0, rp.size - 1, ci.size
    op.row_ptr, op.col_idx, op.val = rp.ctypes.data, ci.ctypes.data, v.ctypes.data
    return op


def stencil_op(nx, ny, nz, kind=N.OP_STENCIL7, faces=None):
    op = N.Operator()
    op.kind, op.ptr_space, op.nx, op.ny, op.nz = kind, 0, nx, ny, nz
    if faces is not None:
        op.kx, op.ky, op.kz = (f.ctypes.data for f in faces)
    return op


ctx = C.c_void_p()
E_ARG, E_UNSUP = 1, 7
rp = np.array([0, 1, 2, 3], np.int32)
ci = np.array([0, 1, 2], np.int32)
v = np.ones(3)
checks = []
# malformed CSR patterns (host arrays are read on the host)
for bad_rp, bad_ci in ((np.array([0, 2, 1, 3], np.int32), ci), (rp, np.array([0, 5, 2], np.int32)),
                       (rp, np.array([0, -1, 2], np.int32)), (np.array([1, 1, 2, 3], np.int32), ci)):
    checks.append(lib.sstep_setup(C.byref(ctx), C.byref(csr_op(bad_rp, bad_ci, v)), 4, 5, 0.1, 1.9, None) == E_ARG)
# bounds, widths, sweeps, NULLs
op = stencil_op(4, 4, 4)
for s, nu, lo, hi in ((0, 5, 0.1, 1.9), (33, 5, 0.1, 1.9), (4, 0, 0.1, 1.9), (4, 5, 1.0, 1.0), (4, 5, -1.0, 1.0),
                      (4, 5, float("nan"), 1.0)):
    checks.append(lib.sstep_setup(C.byref(ctx), C.byref(op), s, nu, lo, hi, None) == E_ARG)
checks.append(lib.sstep_setup(C.byref(ctx), None, 4, 5, 0.1, 1.9, None) == E_ARG)
checks.append(lib.sstep_setup(None, C.byref(op), 4, 5, 0.1, 1.9, None) == E_ARG)
# options
opt = N.Options()
lib.sstep_default_options(C.byref(opt))
opt.gram = 9
checks.append(lib.sstep_setup(C.byref(ctx), C.byref(op), 4, 5, 0.1, 1.9, C.byref(opt)) == E_ARG)
lib.sstep_default_options(C.byref(opt))
opt.gram = N.GRAM_KINDS["recurrence"]
checks.append(lib.sstep_setup(C.byref(ctx), C.byref(op), 32, 5, 0.1, 1.9, C.byref(opt)) == E_UNSUP)
lib.sstep_default_options(C.byref(opt))
opt.basis = 3
checks.append(lib.sstep_setup(C.byref(ctx), C.byref(op), 4, 5, 0.1, 1.9, C.byref(opt)) == E_ARG)
# stencil shapes: partial face arrays, 27-point with coefficients, grid too large
fx = np.ones(5 * 4 * 4)
partial = stencil_op(4, 4, 4)
partial.kx = fx.ctypes.data
checks.append(lib.sstep_setup(C.byref(ctx), C.byref(partial), 4, 5, 0.1, 1.9, None) == E_ARG)
checks.append(lib.sstep_setup(C.byref(ctx), C.byref(stencil_op(4, 4, 4, N.OP_STENCIL27, (fx, fx, fx))), 4, 5, 0.1,
                              1.9, None) == E_ARG)
checks.append(lib.sstep_setup(C.byref(ctx), C.byref(stencil_op(2000, 2000, 2000)), 4, 5, 0.1, 1.9, None) == E_ARG)
# batched and coarse setups
checks.append(lib.sstep_setup_batched(C.byref(ctx), 0, None, 1, 4, 5, None, None, None) == E_ARG)
checks.append(lib.sstep_coarse_setup(C.byref(ctx), C.byref(stencil_op(6, 7, 7)), 0, None) == E_ARG)
# the allocation-free solve's checks before any device work
x = np.zeros(8)
checks.append(lib.sstep_solve_noalloc(C.byref(stencil_op(200, 200, 200, N.OP_STENCIL27)), 32, 20, 0.001, 1.5, None,
                                      x.ctypes.data, x.ctypes.data, 1e-8, None) == E_ARG)
lib.sstep_default_options(C.byref(opt))
opt.precision = 1
checks.append(lib.sstep_solve_noalloc(C.byref(op), 4, 5, 0.1, 1.9, C.byref(opt), x.ctypes.data, x.ctypes.data, 1e-8,
                                      None) == E_UNSUP)
checks.append(lib.sstep_solve_noalloc(C.byref(csr_op(rp, ci, v)), 4, 5, 0.1, 1.9, None, x.ctypes.data,
                                      x.ctypes.data, 1e-8, None) == E_ARG)
# context-free helpers on NULL
checks.append(lib.sstep_solve(None, None, None, 1e-8, None) == E_ARG)
checks.append(lib.sstep_n(None) == 0 and lib.sstep_gram_mode(None) == -1)
for code in range(8):
    lib.sstep_status_string(code)
lib.sstep_destroy(None)
msg = lib.sstep_last_error(None)
assert all(checks), [i for i, c in enumerate(checks) if not c]
print(f"abi exercised: {len(checks)} checks")
