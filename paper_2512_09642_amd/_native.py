"""ctypes declarations of the C ABI in ``include/sstep.h`` (argument
marshalling only).  Loading fails loudly when ``libsstep.so`` has not been
built: there is no fallback implementation."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsstep.so")

SSTEP_OK = 0
STATUS_NAMES = {0: "SSTEP_OK", 1: "SSTEP_E_ARG", 2: "SSTEP_E_HIP", 3: "SSTEP_E_NOMEM", 4: "SSTEP_E_BREAKDOWN",
                5: "SSTEP_E_NOCONV", 6: "SSTEP_E_NONFINITE", 7: "SSTEP_E_UNSUPPORTED"}
OP_CSR, OP_STENCIL7, OP_STENCIL27 = 0, 1, 2
FP64, FP32_IR = 0, 1
GRAM_KINDS = {"auto": 0, "stored": 1, "apply": 2, "recurrence": 3, "moments": 4}
KT_NAMES = ("residual", "basis", "gram", "fgs", "update")

# every symbol the header declares
EXPORTS = (
    "sstep_default_options", "sstep_setup", "sstep_update_coefficients", "sstep_apply", "sstep_solve",
    "sstep_solve_adjoint", "sstep_grad_operator", "sstep_grad_size", "sstep_n", "sstep_step",
    "sstep_lanczos", "sstep_set_bounds", "sstep_lanczos_bounds", "sstep_last_iteration", "sstep_kernel_times", "sstep_gram_mode", "sstep_basis_launches", "sstep_batched_tiles", "sstep_batched_bands", "sstep_setup_batched", "sstep_solve_batched", "sstep_last_error",
    "sstep_status_string", "sstep_destroy", "sstep_solve_noalloc", "sstep_coarse_setup", "sstep_coarse_fgs",
    "sstep_coarse_info",
)


class Operator(C.Structure):
    _fields_ = [("kind", C.c_int32), ("ptr_space", C.c_int32), ("n", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("kx", C.c_void_p), ("ky", C.c_void_p), ("kz", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("precond", C.c_int32), ("p0_mode", C.c_int32),
                ("max_outer", C.c_int32), ("graph_chunk", C.c_int32), ("record_history", C.c_int32),
                ("autotune", C.c_int32), ("gram", C.c_int32), ("basis", C.c_int32), ("basis_steps", C.c_int32),
                ("stream", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("outer_iters", C.c_int32), ("status", C.c_int32), ("rel_res", C.c_double),
                ("res0", C.c_double), ("hist_relres", C.c_void_p), ("hist_delta", C.c_void_p),
                ("hist_cap", C.c_int32), ("hist_lnorm", C.c_void_p)]


class SStepError(RuntimeError):
    """A C-ABI call returned a status other than SSTEP_OK."""

    def __init__(self, status: int, message: str, stats=None):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        self.stats = stats
        super().__init__(f"{self.name}: {message}")


_lib = None


def load():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2512_09642_amd.build` "
                          "(there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    st = C.c_int
    lib.sstep_default_options.argtypes = [C.POINTER(Options)]
    lib.sstep_default_options.restype = None
    lib.sstep_setup.argtypes = [C.POINTER(P), C.POINTER(Operator), C.c_int32, C.c_int32, C.c_double, C.c_double,
                                C.POINTER(Options)]
    lib.sstep_setup.restype = st
    lib.sstep_update_coefficients.argtypes = [P, C.POINTER(Operator)]
    lib.sstep_update_coefficients.restype = st
    lib.sstep_apply.argtypes = [P, P, P]
    lib.sstep_apply.restype = st
    lib.sstep_solve.argtypes = [P, P, P, C.c_double, C.POINTER(Stats)]
    lib.sstep_solve.restype = st
    lib.sstep_solve_adjoint.argtypes = [P, P, P, C.c_double, C.POINTER(Stats)]
    lib.sstep_solve_adjoint.restype = st
    lib.sstep_grad_operator.argtypes = [P, P, P, P, C.c_int32]
    lib.sstep_grad_operator.restype = st
    lib.sstep_grad_size.argtypes = [P]
    lib.sstep_grad_size.restype = C.c_int64
    lib.sstep_n.argtypes = [P]
    lib.sstep_n.restype = C.c_int64
    lib.sstep_step.argtypes = [P, P, P, P, P, P, P, P, P]
    lib.sstep_step.restype = st
    lib.sstep_lanczos.argtypes = [P, P, C.c_int32, P, P, P, P]
    lib.sstep_lanczos.restype = st
    lib.sstep_set_bounds.argtypes = [P, C.c_double, C.c_double]
    lib.sstep_set_bounds.restype = st
    lib.sstep_lanczos_bounds.argtypes = [P, P, C.c_int32, C.c_double, P, P]
    lib.sstep_lanczos_bounds.restype = st
    lib.sstep_last_iteration.argtypes = [P, P, P, P]
    lib.sstep_last_iteration.restype = st
    lib.sstep_kernel_times.argtypes = [P, P, P, C.c_int32, P]
    lib.sstep_kernel_times.restype = st
    lib.sstep_gram_mode.argtypes = [P]
    lib.sstep_gram_mode.restype = C.c_int32
    lib.sstep_basis_launches.argtypes = [P, C.POINTER(C.c_int32)]
    lib.sstep_basis_launches.restype = C.c_int32
    lib.sstep_batched_tiles.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
    lib.sstep_batched_tiles.restype = st
    lib.sstep_batched_bands.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.sstep_batched_bands.restype = st
    lib.sstep_setup_batched.argtypes = [C.POINTER(P), C.c_int32, C.POINTER(Operator), C.c_int32, C.c_int32,
                                        C.c_int32, P, P, C.POINTER(Options)]
    lib.sstep_setup_batched.restype = st
    lib.sstep_solve_batched.argtypes = [P, P, P, C.c_double, P]
    lib.sstep_solve_batched.restype = st
    lib.sstep_solve_noalloc.argtypes = [C.POINTER(Operator), C.c_int32, C.c_int32, C.c_double, C.c_double,
                                        C.POINTER(Options), P, P, C.c_double, C.POINTER(Stats)]
    lib.sstep_solve_noalloc.restype = st
    lib.sstep_coarse_setup.argtypes = [C.POINTER(P), C.POINTER(Operator), C.c_int32, C.POINTER(Options)]
    lib.sstep_coarse_setup.restype = st
    lib.sstep_coarse_fgs.argtypes = [P, P, P, C.c_int32]
    lib.sstep_coarse_fgs.restype = st
    lib.sstep_coarse_info.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.sstep_coarse_info.restype = st
    lib.sstep_last_error.argtypes = [P]
    lib.sstep_last_error.restype = C.c_char_p
    lib.sstep_status_string.argtypes = [C.c_int]
    lib.sstep_status_string.restype = C.c_char_p
    lib.sstep_destroy.argtypes = [P]
    lib.sstep_destroy.restype = None
    _lib = lib
    return lib


def last_error(ctx) -> str:
    msg = load().sstep_last_error(ctx)
    return msg.decode() if msg else ""
