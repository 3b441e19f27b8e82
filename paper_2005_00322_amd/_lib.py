"""ctypes declarations of libpstd's C ABI (include/pstd.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; PSTD_LIBRARY names another build of the same sources (e.g. the host-sanitizer one)
LIB_PATH = os.environ.get("PSTD_LIBRARY") or os.path.join(_PKG, "libpstd.so")

OK = 0
E_INVALID_ARG = -1
E_UNSTABLE = -2
E_UNSUPPORTED = -3
E_HIP = -4
E_OOM = -5
E_NONFINITE = -6

NEUMANN = 0
DIRICHLET = 1
PERIODIC = 2   # both faces of an axis: the Fourier basis, n staggered points
NEUMANN_HALF = 3     # right face half a step beyond the last node (DTT types V-VIII), n staggered points
DIRICHLET_HALF = 4

FP64 = 0
FP32 = 1
SPLIT_BF16 = 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "split_bf16": SPLIT_BF16}


class Grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int64 * 3)]


class State(C.Structure):
    _fields_ = [("p", C.c_void_p), ("u", C.c_void_p * 3), ("step", C.c_int64)]


class NopGate(C.Structure):
    _fields_ = [("validated_error", C.c_double), ("c0_lo", C.c_double), ("c0_hi", C.c_double),
                ("p_max", C.c_double), ("wall_margin", C.c_int32), ("wall_share_max", C.c_double)]


class NopProblem(C.Structure):
    _fields_ = [("dx", C.c_double), ("dt", C.c_double), ("rho0", C.c_double), ("bc", C.c_int32 * 4),
                ("steps", C.c_int64)]


class NopConfig(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("channels", C.c_int32), ("modes", C.c_int32),
                ("layers", C.c_int32), ("hidden", C.c_int32), ("max_batch", C.c_int32), ("split", C.c_int32)]


class PstdError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__("%s: %s (%d): %s" % (where, _STATUS.get(status, "?"), status, detail))
        self.status = status


_STATUS = {OK: "ok", E_INVALID_ARG: "invalid argument", E_UNSTABLE: "unstable", E_UNSUPPORTED: "unsupported",
           E_HIP: "HIP error", E_OOM: "out of memory", E_NONFINITE: "non-finite state"}

_lib = None

# name -> (restype, argtypes)
SIGNATURES = {
    "pstd_plan_create": (C.c_int, [C.POINTER(Grid), C.c_double, C.c_double, C.c_double, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_void_p)]),
    "pstd_plan_create_ex": (C.c_int, [C.POINTER(Grid), C.c_double, C.c_double, C.c_double, C.POINTER(C.c_int32),
                                      C.c_double, C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "pstd_state_init": (C.c_int, [C.c_void_p, C.POINTER(State), C.c_int32]),
    "pstd_step": (C.c_int, [C.c_void_p, C.POINTER(State), C.c_int64]),
    "pstd_step_prepare": (C.c_int, [C.c_void_p, C.POINTER(State), C.c_int64]),
    "pstd_plan_set_path": (C.c_int, [C.c_void_p, C.c_int32]),
    "pstd_apply_axis": (C.c_int, [C.c_void_p, C.POINTER(State), C.c_int32, C.c_int32]),
    "pstd_combine_R": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_int64, C.c_void_p]),
    "pstd_face_weights": (C.c_int, [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "pstd_combine_fields": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.c_double), C.c_int32, C.c_void_p,
                                      C.c_int64, C.c_void_p]),
    "pstd_check_finite": (C.c_int, [C.c_void_p, C.POINTER(State)]),
    "pstd_plan_get_operator": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double)]),
    "pstd_axis_operator": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.c_double, C.c_int32,
                                     C.POINTER(C.c_double)]),
    "pstd_axis_operator_structure": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.c_double, C.c_int32,
                                               C.POINTER(C.c_double), C.POINTER(C.c_double),
                                               C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pstd_apply_axis_operator": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "pstd_plan_numel": (C.c_int64, [C.c_void_p, C.c_int32]),
    "pstd_plan_destroy": (C.c_int, [C.c_void_p]),
    "pstd_batch_create": (C.c_int, [C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double, C.c_void_p,
                                    C.POINTER(C.c_void_p)]),
    "pstd_batch_state_init": (C.c_int, [C.c_void_p, C.POINTER(State), C.c_int32]),
    "pstd_batch_step": (C.c_int, [C.c_void_p, C.POINTER(State), C.c_int64]),
    "pstd_batch_combine_R": (C.c_int, [C.c_void_p, C.POINTER(State), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                       C.POINTER(C.c_void_p), C.c_int32]),
    "pstd_batch_set_config": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]),
    "pstd_batch_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_char_p, C.POINTER(C.c_int32)]),
    "pstd_batch_set_c0_maps": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "pstd_batch_synchronize": (C.c_int, [C.c_void_p]),
    "pstd_batch_destroy": (C.c_int, [C.c_void_p]),
    "pstd_nop_create": (C.c_int, [C.POINTER(NopConfig), C.c_void_p, C.POINTER(C.c_void_p)]),
    "pstd_nop_param_count": (C.c_int64, [C.c_void_p]),
    "pstd_nop_set_params": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "pstd_nop_get_params": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "pstd_nop_get_grads": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "pstd_nop_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "pstd_nop_infer": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "pstd_nop_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "pstd_nop_adam_step": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double]),
    "pstd_nop_relative_errors": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "pstd_nop_input_stats": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "pstd_nop_predict": (C.c_int, [C.c_void_p, C.POINTER(NopGate), C.POINTER(NopProblem), C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_int32, C.c_double, C.c_void_p, C.POINTER(C.c_int32)]),
    "pstd_nop_destroy": (C.c_int, [C.c_void_p]),
    "pstd_relative_errors_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p]),
    "pstd_status_string": (C.c_char_p, [C.c_int]),
    "pstd_last_error": (C.c_char_p, []),
}


def load() -> C.CDLL:
    """Load the in-tree libpstd.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libpstd.so is not built (%s); run `python -m paper_2005_00322_amd.build`" % LIB_PATH)
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != OK:
        detail = load().pstd_last_error()
        raise PstdError(status, where, detail.decode() if detail else "")
