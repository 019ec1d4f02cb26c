"""ctypes declarations of libbfc's C ABI (include/bfc.h)."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbfc.so")

BFC_OK = 0
BFC_EINVAL = 1
BFC_ENOMEM = 2
BFC_EHIP = 3
BFC_ENOTSPD = 4
BFC_ENONFINITE = 5

STATUS_NAMES = {
    BFC_OK: "OK",
    BFC_EINVAL: "EINVAL",
    BFC_ENOMEM: "ENOMEM",
    BFC_EHIP: "EHIP",
    BFC_ENOTSPD: "ENOTSPD",
    BFC_ENONFINITE: "ENONFINITE",
}

BFC_C128 = 0
BFC_C64 = 1
BFC_C64_BF16GRAM = 2
BFC_REG_PROXIMAL = 0
BFC_REG_RIDGE = 1

# every symbol include/bfc.h declares
EXPORTS = (
    "bfc_num_params",
    "bfc_init_cores",
    "bfc_sweep_core",
    "bfc_sweep",
    "bfc_predict_entries",
    "bfc_residual",
    "bfc_get_cores",
    "bfc_set_cores",
    "bfc_sync_status",
    "bfc_destroy",
    "bfc_last_error",
    "bfc_profile_enable",
    "bfc_profile_read",
    "bfc_core_stats",
    "bfc_solve_counters",
    "bfc_residual_observed",
    "bfc_relative_error",
    "bfc_relative_error_observed",
    "bfc_use_graphs",
    "bfc_batch_create",
    "bfc_batch_sweep",
    "bfc_batch_residuals",
    "bfc_batch_destroy",
    "bfc_set_item_size",
    "bfc_autotune_item_size",
    "bfc_lowrank_to_butterfly",
    "bfc_validate",
    "bfc_debug_fail_allocation_after",
    "bfc_lowrank_to_butterfly_noalloc",
    "bfc_adam_sweep",
    "bfc_adam_reset",
    "bfc_adf_sweep",
    "bfc_set_cores_f32",
    "bfc_set_values",
    "bfc_loss_gradient",
    "bfc_loss_gradient_batch",
    "bfc_mlp_forward",
    "bfc_mlp_backward",
    "bfc_mlp_forward_bf16",
    "bfc_mlp_to_bf16",
    "bfc_mlp_adam",
)

KERNEL_KINDS = {"outer": 0, "inner_gram": 1, "inner_solve": 2, "residual": 3, "predict": 4,
                "env": 5, "inner_ir": 6}


class BfcConfig(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("L", ctypes.c_int32),
        ("r", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("reg_mode", ctypes.c_int32),
        ("reg_rel", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("reg_floor", ctypes.c_double),
    ]


_lib = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Load libbfc.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    P = ctypes.c_void_p
    lib.bfc_num_params.argtypes = [i64, i32, i32]
    lib.bfc_num_params.restype = i64
    lib.bfc_init_cores.argtypes = [ctypes.POINTER(BfcConfig), i64, vp, vp, vp, vp, vp,
                                   ctypes.POINTER(P)]
    lib.bfc_init_cores.restype = i32
    lib.bfc_sweep_core.argtypes = [P, i32, vp]
    lib.bfc_sweep_core.restype = i32
    lib.bfc_sweep.argtypes = [P, vp]
    lib.bfc_sweep.restype = i32
    lib.bfc_predict_entries.argtypes = [P, i64, vp, vp, vp, vp]
    lib.bfc_predict_entries.restype = i32
    lib.bfc_residual.argtypes = [P, i64, vp, vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.bfc_relative_error.argtypes = [P, i64, vp, vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.bfc_relative_error.restype = i32
    lib.bfc_relative_error_observed.argtypes = [P, ctypes.POINTER(ctypes.c_double), vp]
    lib.bfc_relative_error_observed.restype = i32
    lib.bfc_residual.restype = i32
    lib.bfc_get_cores.argtypes = [P, vp, vp]
    lib.bfc_get_cores.restype = i32
    lib.bfc_set_cores.argtypes = [P, vp, vp]
    lib.bfc_set_cores.restype = i32
    lib.bfc_sync_status.argtypes = [P, vp]
    lib.bfc_sync_status.restype = i32
    lib.bfc_destroy.argtypes = [P]
    lib.bfc_destroy.restype = None
    lib.bfc_profile_enable.argtypes = [P, i32]
    lib.bfc_profile_enable.restype = i32
    lib.bfc_profile_read.argtypes = [P, i32, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64)]
    lib.bfc_profile_read.restype = i32
    lib.bfc_core_stats.argtypes = [P, i32, ctypes.POINTER(ctypes.c_int64)]
    lib.bfc_core_stats.restype = i32
    lib.bfc_solve_counters.argtypes = [P, i32, ctypes.POINTER(ctypes.c_int64), vp]
    lib.bfc_solve_counters.restype = i32
    lib.bfc_residual_observed.argtypes = [P, ctypes.POINTER(ctypes.c_double), vp]
    lib.bfc_residual_observed.restype = i32
    lib.bfc_use_graphs.argtypes = [P, i32]
    lib.bfc_use_graphs.restype = i32
    lib.bfc_batch_create.argtypes = [ctypes.POINTER(P), i32, ctypes.POINTER(P)]
    lib.bfc_batch_create.restype = i32
    lib.bfc_batch_sweep.argtypes = [P, vp]
    lib.bfc_batch_sweep.restype = i32
    lib.bfc_batch_residuals.argtypes = [P, ctypes.POINTER(ctypes.c_double), vp]
    lib.bfc_batch_residuals.restype = i32
    lib.bfc_batch_destroy.argtypes = [P]
    lib.bfc_batch_destroy.restype = i32
    lib.bfc_set_item_size.argtypes = [P, i32, vp]
    lib.bfc_set_item_size.restype = i32
    lib.bfc_autotune_item_size.argtypes = [ctypes.POINTER(P), i32, i32, ctypes.POINTER(i32), i32,
                                           ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                                           vp]
    lib.bfc_autotune_item_size.restype = i32
    lib.bfc_lowrank_to_butterfly.argtypes = [i64, i32, i32, i32, i32, vp, vp, vp, vp, vp]
    lib.bfc_lowrank_to_butterfly.restype = i32
    lib.bfc_validate.argtypes = [P]
    lib.bfc_validate.restype = i32
    lib.bfc_debug_fail_allocation_after.argtypes = [i64]
    lib.bfc_debug_fail_allocation_after.restype = i64
    lib.bfc_lowrank_to_butterfly_noalloc.argtypes = [i64, i32, i32, i32, i32, vp, vp, vp, vp, vp]
    lib.bfc_lowrank_to_butterfly_noalloc.restype = i32
    d = ctypes.c_double
    lib.bfc_adam_sweep.argtypes = [P, i32, d, d, d, d, vp]
    lib.bfc_adam_sweep.restype = i32
    lib.bfc_adam_reset.argtypes = [P, vp]
    lib.bfc_adam_reset.restype = i32
    lib.bfc_adf_sweep.argtypes = [P, vp]
    lib.bfc_adf_sweep.restype = i32
    lib.bfc_set_cores_f32.argtypes = [P, vp, vp]
    lib.bfc_set_cores_f32.restype = i32
    lib.bfc_set_values.argtypes = [P, vp, vp]
    lib.bfc_set_values.restype = i32
    f = ctypes.c_float
    lib.bfc_loss_gradient.argtypes = [P, f, vp, i32, ctypes.POINTER(ctypes.c_double), vp]
    lib.bfc_loss_gradient.restype = i32
    lib.bfc_loss_gradient_batch.argtypes = [P, i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                            ctypes.POINTER(f), ctypes.POINTER(vp), i32,
                                            ctypes.POINTER(ctypes.c_double), vp]
    lib.bfc_loss_gradient_batch.restype = i32
    lib.bfc_mlp_forward.argtypes = [i64, i64, i64, vp, vp, vp, i32, vp, vp]
    lib.bfc_mlp_forward.restype = i32
    lib.bfc_mlp_backward.argtypes = [i64, i64, i64, vp, vp, vp, vp, i32, vp, vp, vp, vp]
    lib.bfc_mlp_backward.restype = i32
    lib.bfc_mlp_forward_bf16.argtypes = [i64, i64, i64, vp, vp, vp, i32, vp, vp, vp]
    lib.bfc_mlp_forward_bf16.restype = i32
    lib.bfc_mlp_to_bf16.argtypes = [i64, vp, vp, vp]
    lib.bfc_mlp_to_bf16.restype = i32
    lib.bfc_mlp_adam.argtypes = [i64, vp, vp, vp, vp, i32, f, f, f, f, vp]
    lib.bfc_mlp_adam.restype = i32
    lib.bfc_last_error.argtypes = []
    lib.bfc_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib
