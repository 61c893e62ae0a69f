"""ctypes binding of libvlb.so (include/vlb.h).  Argument marshalling only.

The library is loaded from this package directory.  If it is missing the import of
any simulation object fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# VLB_LIBRARY selects another in-tree build of the same library (tuning variants).
LIB_PATH = os.environ.get("VLB_LIBRARY") or os.path.join(PKG, "libvlb.so")

VLB_OK = 0
VLB_E_INVALID_ARG = -1
VLB_E_WORKSPACE = -2
VLB_E_HIP = -3
VLB_E_NONFINITE = -4
VLB_E_STATE = -5
VLB_E_UNSUPPORTED = -6
VLB_FP32, VLB_FP64 = 0, 1
VLB_PERIODIC, VLB_WALL, VLB_OPEN, VLB_WET = 0, 1, 2, 3
VLB_FLAG_NO_SOURCE = 1
VLB_FLAG_CURVED_YLW = 2
VLB_FLAG_OPEN_NEBB = 4
MODES = {"periodic": VLB_PERIODIC, "wall": VLB_WALL, "open": VLB_OPEN, "wet": VLB_WET}

# Every symbol declared in include/vlb.h.
EXPORTS = [
    "vlb_create", "vlb_destroy", "vlb_workspace_bytes", "vlb_geometry", "vlb_bind",
    "vlb_set_params", "vlb_set_force_field", "vlb_set_inlet", "vlb_init_equilibrium",
    "vlb_step", "vlb_get_step", "vlb_read_fields", "vlb_read_history", "vlb_monitors",
    "vlb_drag",
    "vlb_state_bytes", "vlb_save_state", "vlb_load_state", "vlb_set_tile",
    "vlb_set_store_mode", "vlb_set_graph_chunk", "vlb_set_schedule", "vlb_adjoint_workspace_bytes",
    "vlb_adjoint_forward", "vlb_adjoint_backward", "vlb_adjoint", "vlb_batch_workspace_bytes",
    "vlb_batch_create", "vlb_batch_create_noalloc", "vlb_batch_step", "vlb_batch_read_fields", "vlb_batch_set_graph_chunk",
    "vlb_batch_set_persistent", "vlb_batch_set_schedule",
    "vlb_batch_destroy", "vlb_params_from_groups",
    "vlb_error_string", "vlb_last_error_detail",
]
# Every symbol declared in include/vlb3d.h (the three-dimensional D3Q19 form).
EXPORTS3 = [
    "vlb3_create", "vlb3_workspace_bytes", "vlb3_bind", "vlb3_set_params",
    "vlb3_init_equilibrium", "vlb3_step", "vlb3_read_fields", "vlb3_get_step", "vlb3_destroy",
    "vlb3_set_solid", "vlb3_set_closure",
]


class VlbGrid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("xmode", C.c_int), ("ymode", C.c_int),
                ("precision", C.c_int), ("solid_mask", C.c_void_p),
                ("circles", C.POINTER(C.c_double)), ("ncircles", C.c_int)]


class VlbParams(C.Structure):
    _fields_ = [("nu_s", C.c_double), ("eta_p", C.c_double), ("lambda_", C.c_double),
                ("kappa", C.c_double), ("Lambda_s", C.c_double), ("Lambda_p", C.c_double),
                ("Fx", C.c_double), ("Fy", C.c_double), ("flags", C.c_int),
                ("model", C.c_int), ("model_param", C.c_double)]


# constitutive closures (VLB_OLDROYD_B ... VLB_FENE_P) by name
MODELS = {"oldroyd_b": 0, "giesekus": 1, "lptt": 2, "eptt": 3, "fene_p": 4}


class VlbMonitor(C.Structure):
    _fields_ = [("mass", C.c_double * 4), ("residual", C.c_double), ("umax", C.c_double),
                ("step", C.c_int64), ("nonfinite", C.c_int64), ("spd_violations", C.c_int64)]


class VlbError(RuntimeError):
    def __init__(self, status, where, detail):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


_lib = None


def load():
    """Load libvlb.so from the package directory (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2508_16997_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    I = C.c_int
    lib.vlb_create.argtypes = [C.POINTER(VlbGrid), C.POINTER(P)]
    lib.vlb_destroy.argtypes = [P]
    lib.vlb_destroy.restype = None
    lib.vlb_workspace_bytes.argtypes = [P, C.POINTER(C.c_size_t)]
    lib.vlb_geometry.argtypes = [P, P, P, P, P, I, C.POINTER(I)]
    lib.vlb_bind.argtypes = [P, P, C.c_size_t, P]
    lib.vlb_set_params.argtypes = [P, C.POINTER(VlbParams)]
    lib.vlb_set_force_field.argtypes = [P, P, P]
    lib.vlb_set_inlet.argtypes = [P, P, P, P, P]
    lib.vlb_init_equilibrium.argtypes = [P, P, P, P, P, P, P]
    lib.vlb_step.argtypes = [P, C.c_int64]
    lib.vlb_get_step.argtypes = [P, C.POINTER(C.c_int64)]
    lib.vlb_read_fields.argtypes = [P, P, P, P, P, P, P]
    lib.vlb_read_history.argtypes = [P, P, P, P, P, P]
    lib.vlb_monitors.argtypes = [P, C.POINTER(VlbMonitor)]
    lib.vlb_state_bytes.argtypes = [P, C.POINTER(C.c_size_t)]
    lib.vlb_save_state.argtypes = [P, P, C.c_size_t]
    lib.vlb_load_state.argtypes = [P, P, C.c_size_t]
    lib.vlb_set_tile.argtypes = [P, I]
    lib.vlb_set_graph_chunk.argtypes = [P, I]
    lib.vlb_set_store_mode.argtypes = [P, I]
    lib.vlb_set_schedule.argtypes = [P, I, I]
    lib.vlb_drag.argtypes = [P, I, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    D = C.POINTER(C.c_double)
    lib.vlb_adjoint_workspace_bytes.argtypes = [P, C.c_int64, I, C.POINTER(C.c_size_t)]
    lib.vlb_adjoint_forward.argtypes = [P, C.c_int64, I, P, C.c_size_t]
    lib.vlb_adjoint_backward.argtypes = [P, P, P, D, D, P, P, P, C.c_size_t]
    lib.vlb_adjoint.argtypes = [P, C.c_int64, I, P, P, D, D, D, P, P, P, C.c_size_t]
    lib.vlb_batch_workspace_bytes.argtypes = [P, I, I, C.POINTER(C.c_size_t)]
    lib.vlb_batch_create.argtypes = [P, I, I, P, C.c_size_t, C.POINTER(P)]
    lib.vlb_batch_create_noalloc.argtypes = [P, I, I, C.POINTER(P)]
    lib.vlb_batch_step.argtypes = [P, C.c_int64]
    lib.vlb_batch_set_graph_chunk.argtypes = [P, I]
    lib.vlb_batch_set_persistent.argtypes = [P, I]
    lib.vlb_batch_set_schedule.argtypes = [P, I, I]
    lib.vlb_batch_read_fields.argtypes = [P, I, P, P, P, P, P, P]
    Dd = C.c_double
    lib.vlb_params_from_groups.argtypes = [Dd, Dd, Dd, Dd, Dd, Dd, Dd, Dd,
                                           C.POINTER(VlbParams), C.POINTER(Dd)]
    lib.vlb_batch_destroy.argtypes = [P]
    lib.vlb_batch_destroy.restype = None
    lib.vlb_error_string.argtypes = [I]
    lib.vlb_error_string.restype = C.c_char_p
    lib.vlb_last_error_detail.argtypes = []
    lib.vlb_last_error_detail.restype = C.c_char_p
    for name in EXPORTS + EXPORTS3:
        if name not in ("vlb_destroy", "vlb_batch_destroy", "vlb_error_string",
                        "vlb_last_error_detail", "vlb3_destroy"):
            getattr(lib, name).restype = I
    D = C.c_double
    PA = C.POINTER(C.c_void_p)
    lib.vlb3_create.argtypes = [I, I, I, I, I, I, C.POINTER(P)]
    lib.vlb3_set_solid.argtypes = [P, C.c_void_p]
    lib.vlb3_set_closure.argtypes = [P, I, D]
    lib.vlb3_workspace_bytes.argtypes = [P, C.POINTER(C.c_size_t)]
    lib.vlb3_bind.argtypes = [P, P, C.c_size_t, P]
    lib.vlb3_set_params.argtypes = [P, D, D, D, D, D, D, D, D, D, I]
    lib.vlb3_init_equilibrium.argtypes = [P, PA]
    lib.vlb3_step.argtypes = [P, C.c_int64]
    lib.vlb3_read_fields.argtypes = [P, PA]
    lib.vlb3_get_step.argtypes = [P, C.POINTER(C.c_int64)]
    lib.vlb3_destroy.argtypes = [P]
    lib.vlb3_destroy.restype = None
    _lib = lib
    return lib


def check(status, where):
    if status != VLB_OK:
        lib = load()
        detail = lib.vlb_last_error_detail().decode(errors="replace")
        raise VlbError(status, where, detail or lib.vlb_error_string(status).decode())
    return status
