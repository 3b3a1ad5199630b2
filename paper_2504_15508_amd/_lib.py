"""ctypes loader of libdplr_lr.so (the C ABI in include/dplr_lr.h).

There is no fallback: if the shared library is missing or fails to load, the
import raises, so nothing silently runs elsewhere."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdplr_lr.so")

OK, E_INVALID, E_UNSUPPORTED, E_NO_BOX, E_CAPACITY, E_DEVICE, E_NOMEM = range(7)
STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_UNSUPPORTED", 3: "E_NO_BOX", 4: "E_CAPACITY",
                5: "E_DEVICE", 6: "E_NOMEM"}
FP32, FP64 = 0, 1
ACCUMULATE, NO_VIRIAL, DIFF_AD = 0x1, 0x2, 0x4
BUF_SPECTRUM, BUF_INFLUENCE, BUF_FIELD_SPECTRA, BUF_Q32_CLAMPED = 0, 1, 2, 3
NOALLOC_SCRATCH_BYTES = 128 << 20  # DPLR_LR_NOALLOC_SCRATCH_BYTES

# every symbol include/dplr_lr.h declares
EXPORTS = [
    "dplr_lr_abi_version", "dplr_lr_config_default", "dplr_lr_config_validate",
    "dplr_lr_plan_create", "dplr_lr_set_stream", "dplr_lr_set_fft_int32", "dplr_lr_set_box",
    "dplr_lr_compute_energy_forces_virial", "dplr_lr_compute_noalloc", "dplr_lr_scale_grad",
    "dplr_lr_plan_destroy",
    "dplr_lr_last_error", "dplr_lr_workspace_bytes", "dplr_lr_debug_copy", "dplr_lr_debug_size",
    "dplr_lr_debug_dft_q32",
    "dplr_lr_profile_enable", "dplr_lr_profile_read", "dplr_lr_profile_stage_name",
    "dplr_lr_mlp_config_default", "dplr_lr_mlp_param_count", "dplr_lr_mlp_create", "dplr_lr_mlp_destroy",
    "dplr_lr_mlp_set_stream", "dplr_lr_mlp_set_params", "dplr_lr_mlp_get_params",
    "dplr_lr_mlp_state_bytes", "dplr_lr_mlp_get_state", "dplr_lr_mlp_set_state", "dplr_lr_mlp_forward",
    "dplr_lr_mlp_train_step", "dplr_lr_mlp_descriptor", "dplr_lr_mlp_last_error", "dplr_lr_guard_decide",
    "dplr_lr_mlp_norm_accumulate", "dplr_lr_mlp_norm_finish", "dplr_lr_mlp_set_train_charges",
    "dplr_lr_mlp_check_charges", "dplr_lr_mlp_audit", "dplr_lr_mlp_read_stats",
]
GUARD_LEARNED, GUARD_FINE, GUARD_AUDIT = 0, 1, 2


class MlpConfig(ctypes.Structure):
    _fields_ = [("cutoff", ctypes.c_double), ("out_scale", ctypes.c_double), ("capacity", ctypes.c_int64),
                ("flags", ctypes.c_uint32)]


class GuardConfig(ctypes.Structure):
    _fields_ = [("max_audit_rel_rmse", ctypes.c_double), ("max_correction_ratio", ctypes.c_double),
                ("audit_interval", ctypes.c_int64), ("min_neighbours", ctypes.c_double),
                ("max_neighbours", ctypes.c_double)]


class GuardStats(ctypes.Structure):
    _fields_ = [("audit_valid", ctypes.c_int32), ("audit_rel_rmse", ctypes.c_double),
                ("steps_since_audit", ctypes.c_int64), ("max_correction", ctypes.c_double),
                ("max_force", ctypes.c_double), ("min_neighbours", ctypes.c_double),
                ("max_neighbours", ctypes.c_double), ("unseen_charges", ctypes.c_int32)]


class Config(ctypes.Structure):
    _fields_ = [("mesh", ctypes.c_int32 * 3), ("order", ctypes.c_int32), ("beta", ctypes.c_double),
                ("coulomb_k", ctypes.c_double), ("precision", ctypes.c_int32),
                ("alias_range", ctypes.c_int32), ("capacity", ctypes.c_int64), ("flags", ctypes.c_uint32)]


class DplrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          "python paper_2504_15508_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    p, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    cfgp = ctypes.POINTER(Config)
    sig = {
        "dplr_lr_abi_version": ([], i32),
        "dplr_lr_config_default": ([cfgp], None),
        "dplr_lr_config_validate": ([cfgp, ctypes.c_char_p, i64], ctypes.c_int),
        "dplr_lr_plan_create": ([cfgp, p, ctypes.POINTER(p)], ctypes.c_int),
        "dplr_lr_set_stream": ([p, p], ctypes.c_int),
        "dplr_lr_set_fft_int32": ([p, ctypes.POINTER(i32), d], ctypes.c_int),
        "dplr_lr_set_box": ([p, ctypes.POINTER(d)], ctypes.c_int),
        "dplr_lr_compute_energy_forces_virial": ([p, i64, p, p, i64, p, p, p, p, p, p], ctypes.c_int),
        "dplr_lr_compute_noalloc": ([cfgp, ctypes.POINTER(d), i64, p, p, i64, p, p, p, p, p, p, p], ctypes.c_int),
        "dplr_lr_scale_grad": ([p, p, i64, p, p, i64, p, p], ctypes.c_int),
        "dplr_lr_plan_destroy": ([p], ctypes.c_int),
        "dplr_lr_last_error": ([p], ctypes.c_char_p),
        "dplr_lr_workspace_bytes": ([p], i64),
        "dplr_lr_debug_copy": ([p, i32, p, i64], ctypes.c_int),
        "dplr_lr_debug_size": ([p, i32], i64),
        "dplr_lr_debug_dft_q32": ([p, i32, i32, p, i32], ctypes.c_int),
        "dplr_lr_profile_enable": ([p, i32], ctypes.c_int),
        "dplr_lr_profile_read": ([p, p, p, i32, p, i32], ctypes.c_int),
        "dplr_lr_profile_stage_name": ([i32], ctypes.c_char_p),
        "dplr_lr_mlp_config_default": ([ctypes.POINTER(MlpConfig)], None),
        "dplr_lr_mlp_param_count": ([], i64),
        "dplr_lr_mlp_create": ([ctypes.POINTER(MlpConfig), p, ctypes.POINTER(p)], ctypes.c_int),
        "dplr_lr_mlp_destroy": ([p], ctypes.c_int),
        "dplr_lr_mlp_set_stream": ([p, p], ctypes.c_int),
        "dplr_lr_mlp_set_params": ([p, p, i64], ctypes.c_int),
        "dplr_lr_mlp_get_params": ([p, p, i64], ctypes.c_int),
        "dplr_lr_mlp_state_bytes": ([], i64),
        "dplr_lr_mlp_get_state": ([p, p, i64], ctypes.c_int),
        "dplr_lr_mlp_set_state": ([p, p, i64], ctypes.c_int),
        "dplr_lr_mlp_forward": ([p, ctypes.POINTER(d), i64, p, p, i64, p, p, p, p, i32], ctypes.c_int),
        "dplr_lr_mlp_train_step": ([p, ctypes.POINTER(d), i64, p, p, i64, p, p, p, p, p, p, ctypes.c_float, p, p],
                                   ctypes.c_int),
        "dplr_lr_mlp_norm_accumulate": ([p, ctypes.POINTER(d), i64, p, p, i64, p, p], ctypes.c_int),
        "dplr_lr_mlp_norm_finish": ([p], ctypes.c_int),
        "dplr_lr_mlp_set_train_charges": ([p, p, i32], ctypes.c_int),
        "dplr_lr_mlp_check_charges": ([p, i64, p, i64, p], ctypes.c_int),
        "dplr_lr_mlp_audit": ([p, i64, p, p, i64, p, p, i32], ctypes.c_int),
        "dplr_lr_mlp_read_stats": ([p, ctypes.POINTER(GuardStats)], ctypes.c_int),
        "dplr_lr_mlp_descriptor": ([p, ctypes.POINTER(d), i64, p, p, i64, p, p, p, p], ctypes.c_int),
        "dplr_lr_mlp_last_error": ([p], ctypes.c_char_p),
        "dplr_lr_guard_decide": ([ctypes.POINTER(GuardConfig), ctypes.POINTER(GuardStats), ctypes.POINTER(i32)],
                                 ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def check(status: int, plan_handle=None):
    if status != OK:
        msg = load().dplr_lr_last_error(plan_handle)
        raise DplrError(status, msg.decode() if msg else "")


def check_mlp(status: int, handle=None):
    if status != OK:
        msg = load().dplr_lr_mlp_last_error(handle)
        raise DplrError(status, msg.decode() if msg else "")
