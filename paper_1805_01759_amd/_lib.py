"""ctypes binding of libl1ls.so (include/l1ls.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libl1ls.so")

L1LS_FP32 = 0
L1LS_SPLIT_BF16 = 1

PX_CONVERGED = 1
PX_MAX_ITER = 2
PX_NONFINITE = 4
PX_POLISHED = 8
PX_ZERO = 16
PX_BAD_LAMBDA = 32

STATUS_NAMES = {0: "L1LS_OK", -1: "L1LS_ERR_INVALID_ARG", -2: "L1LS_ERR_UNSUPPORTED_SHAPE",
                -3: "L1LS_ERR_WORKSPACE", -4: "L1LS_ERR_HIP", -5: "L1LS_ERR_INTERNAL"}

EXPORTS = [
    "l1ls_options_default", "l1ls_workspace_size", "l1ls_solve", "l1ls_solve_noalloc",
    "l1ls_solve_blocks",
    "l1ls_plan_create", "l1ls_plan_workspace_size", "l1ls_plan_execute", "l1ls_plan_destroy",
    "l1ls_plan_describe",
    "l1ls_unrolled_tape_size", "l1ls_unrolled_backward_ws_size", "l1ls_unrolled_forward",
    "l1ls_unrolled_backward", "l1ls_status_string", "l1ls_last_error",
    "l1ls_timing_enable", "l1ls_timing_read", "l1ls_timing_read_kernel", "l1ls_solve_counters",
    "l1ls_solve_constants",
]

# kernel classes for l1ls_timing_read_kernel
KERNEL_ITERATION, KERNEL_REFINE, KERNEL_CERTIFY = 0, 1, 2

# L1LS_NOALLOC_SCRATCH_BYTES: the fixed scratch of l1ls_solve_noalloc
NOALLOC_SCRATCH_BYTES = 64 << 20


class Options(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("tol", ctypes.c_float), ("c_alpha", ctypes.c_float),
                ("precision", ctypes.c_int32), ("backtracking", ctypes.c_int32),
                ("monotone", ctypes.c_int32), ("fp64_polish", ctypes.c_int32),
                ("polish_after", ctypes.c_int32), ("warm_start", ctypes.c_int32),
                ("fp64_continue", ctypes.c_int32),
                ("iteration_kernel", ctypes.c_int32)]


class Diag(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_void_p), ("kkt", ctypes.c_void_p), ("objective", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("nnz", ctypes.c_void_p)]


class Stack(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("l", ctypes.c_int32), ("p", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("lambda_", ctypes.c_void_p),
                ("lambda_stride", ctypes.c_int64), ("X", ctypes.c_void_p), ("diag", Diag)]


_lib = None


class L1LSError(RuntimeError):
    pass


def load() -> ctypes.CDLL:
    """Load the in-tree HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO_PATH):
        raise L1LSError(f"{SO_PATH} is missing: build it with `python -m paper_1805_01759_amd.build`")
    L = ctypes.CDLL(SO_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    st = ctypes.c_int
    L.l1ls_options_default.argtypes = []
    L.l1ls_options_default.restype = Options
    L.l1ls_workspace_size.argtypes = [I32, I32, I64, ctypes.POINTER(Options), ctypes.POINTER(SZ)]
    L.l1ls_workspace_size.restype = st
    L.l1ls_solve.argtypes = [I32, I32, I64, P, P, P, I64, ctypes.POINTER(Options), P,
                             ctypes.POINTER(Diag), P, SZ, P]
    L.l1ls_solve.restype = st
    L.l1ls_solve_noalloc.argtypes = [I32, I32, I64, P, P, P, I64, ctypes.POINTER(Options), P,
                                     ctypes.POINTER(Diag), P]
    L.l1ls_solve_noalloc.restype = st
    L.l1ls_solve_blocks.argtypes = [I32, I32, I64, P, P, P, I64, ctypes.POINTER(Options), I32, P, P,
                                    ctypes.POINTER(Diag), P, ctypes.c_size_t, P]
    L.l1ls_solve_blocks.restype = st
    L.l1ls_plan_create.argtypes = [ctypes.POINTER(Stack), I32, ctypes.POINTER(Options),
                                   ctypes.POINTER(P)]
    L.l1ls_plan_create.restype = st
    L.l1ls_plan_workspace_size.argtypes = [P, ctypes.POINTER(SZ)]
    L.l1ls_plan_workspace_size.restype = st
    L.l1ls_plan_execute.argtypes = [P, ctypes.POINTER(Stack), P, SZ, P]
    L.l1ls_plan_execute.restype = st
    L.l1ls_plan_destroy.argtypes = [P]
    L.l1ls_plan_destroy.restype = None
    L.l1ls_plan_describe.argtypes = [P, ctypes.c_char_p, I32]
    L.l1ls_plan_describe.restype = I32
    L.l1ls_unrolled_tape_size.argtypes = [I32, I32, I64, I32, I32, ctypes.POINTER(SZ)]
    L.l1ls_unrolled_tape_size.restype = st
    L.l1ls_unrolled_backward_ws_size.argtypes = [I32, I32, I64, I32, I32, ctypes.POINTER(SZ)]
    L.l1ls_unrolled_backward_ws_size.restype = st
    L.l1ls_unrolled_forward.argtypes = [I32, I32, I64, P, P, P, ctypes.c_float, ctypes.c_float,
                                        I32, I32, P, P, SZ, P]
    L.l1ls_unrolled_forward.restype = st
    L.l1ls_unrolled_backward.argtypes = [I32, I32, I64, P, P, P, ctypes.c_float, ctypes.c_float,
                                         I32, I32, P, SZ, P, P, P, P, P, SZ, P]
    L.l1ls_unrolled_backward.restype = st
    L.l1ls_status_string.argtypes = [st]
    L.l1ls_status_string.restype = ctypes.c_char_p
    L.l1ls_last_error.argtypes = []
    L.l1ls_last_error.restype = ctypes.c_char_p
    L.l1ls_timing_enable.argtypes = [I32]
    L.l1ls_timing_enable.restype = None
    L.l1ls_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I32)]
    L.l1ls_timing_read.restype = I32
    L.l1ls_timing_read_kernel.argtypes = [I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I32)]
    L.l1ls_timing_read_kernel.restype = I32
    L.l1ls_solve_counters.argtypes = [I32, I32, I64, P, P, ctypes.POINTER(ctypes.c_uint64 * 5)]
    L.l1ls_solve_counters.restype = st
    L.l1ls_solve_constants.argtypes = [I32, I32, I64, P, P, ctypes.POINTER(ctypes.c_double * 3)]
    L.l1ls_solve_constants.restype = st
    _lib = L
    return L


def check(status: int, what: str = "l1ls") -> None:
    if status != 0:
        detail = load().l1ls_last_error().decode()
        raise L1LSError(f"{what}: {STATUS_NAMES.get(status, status)}: {detail}")
