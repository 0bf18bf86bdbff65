"""ctypes declarations of the C ABI in include/ib.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libibwave.so")

IB_OK = 0
IB_ERR_ARG, IB_ERR_HIP, IB_ERR_OOM, IB_ERR_UNCONSTRAINED, IB_ERR_NONFINITE, IB_ERR_STATE = -1, -2, -3, -4, -5, -6
IB_F32, IB_F64 = 0, 1
IB_SURF_FREE, IB_SURF_RIGID, IB_SURF_ROBIN = 0, 1, 2
IB_FORM_P2 = 0
IB_FORM_PV1 = 1
IB_METHOD_ND = 0
IB_METHOD_1D = 1
FIELD_NODE_CLASS, FIELD_BPOINTS, FIELD_IB_NODES, FIELD_IB_META, FIELD_WEIGHTS_F64, FIELD_SIGMA = range(6)
FIELD_PV_ROWS, FIELD_PV_ENTRIES, FIELD_VCLASS = 6, 7, 8
FIELD_BC_COUNTS, FIELD_BC_ENTRIES = 9, 10


class ib_grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("reserved", C.c_int32), ("n", C.c_int64 * 3), ("h", C.c_double)]


class ib_params(C.Structure):
    _fields_ = [("form", C.c_int32), ("surface", C.c_int32), ("space_order", C.c_int32),
                ("max_radius_steps", C.c_int32), ("min_basis_order", C.c_int32), ("physical_below", C.c_int32),
                ("eta", C.c_double), ("rank_rtol", C.c_double), ("eta_v", C.c_double), ("method", C.c_int32),
                ("keep_bc_weights", C.c_int32), ("robin_dev", C.c_void_p)]


class ib_stats(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_interior", C.c_int64), ("n_boundary_points", C.c_int64),
                ("n_ib", C.c_int64), ("sum_nw", C.c_int64), ("max_nw", C.c_int64),
                ("radius_hist", C.c_int64 * 8), ("order_hist", C.c_int64 * 17), ("max_cond", C.c_double),
                ("min_margin", C.c_double), ("table_bytes_f32", C.c_int64), ("table_bytes_f64", C.c_int64),
                ("max_ball", C.c_int64), ("build_ms", C.c_double), ("dense_weights", C.c_int64),
                ("col_weights", C.c_int64)]


EXPORTS = {
    "ib_abi_version": (C.c_int32, []),
    "ib_last_error": (C.c_char_p, []),
    "ib_build_weights": (C.c_int, [C.POINTER(ib_grid), C.c_void_p, C.POINTER(ib_params), C.c_void_p,
                                   C.POINTER(C.c_void_p)]),
    "ib_weights_stats": (C.c_int, [C.c_void_p, C.POINTER(ib_stats)]),
    "ib_weights_free": (None, [C.c_void_p]),
    "ib_weights_copy": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64]),
    "ib_state_create": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_double, C.c_int32,
                                  C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                  C.POINTER(C.c_void_p)]),
    "ib_state_free": (None, [C.c_void_p]),
    "ib_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p]),
    "ib_forward": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p]),
    "ib_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "ib_adjoint_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "ib_forward_ckpt": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32,
                                  C.POINTER(C.c_void_p), C.c_void_p]),
    "ib_adjoint_ckpt": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                  C.c_void_p]),
    "ib_checkpoints_free": (None, [C.c_void_p]),
    "ib_state_set_watchdog": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_void_p]),
    "ib_state_status": (C.c_int, [C.c_void_p, C.c_int32]),
    "ib_state_field": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p]),
    "ib_state_step_count": (C.c_int64, [C.c_void_p]),
    "ib_state_set_tuning": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]),
    "ib_state_run_kernel": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "ib_state_set_forcing": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p]),
}

_lib = None


def load():
    """Load the built library; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_2309_03600_amd.build.build() first")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


class NonFiniteError(RuntimeError):
    """The watchdog found a non-finite or oversized pressure (IB_ERR_NONFINITE)."""


def check(status):
    if status != IB_OK:
        msg = load().ib_last_error()
        text = f"ibwave error {status}: {msg.decode() if msg else ''}"
        raise (NonFiniteError if status == IB_ERR_NONFINITE else RuntimeError)(text)
