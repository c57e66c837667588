"""ctypes binding of libpermgpu.so (the C ABI in include/perm.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  If the library has not been built, importing this module raises
ImportError -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpermgpu.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python paper_2510_03421_amd/build.py or __graft_entry__.build())")

lib = ctypes.CDLL(LIB_PATH)

# enums of perm.h
PERM_OK, PERM_E_INVALID, PERM_E_TOO_LARGE, PERM_E_OVERFLOW, PERM_E_HIP, PERM_E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5
PERM_F64, PERM_C128, PERM_I64, PERM_B8 = 0, 1, 2, 3
PERM_OUT_F64, PERM_OUT_C128, PERM_OUT_I64, PERM_OUT_I128, PERM_OUT_DD, PERM_OUT_CDD = \
    0, 1, 2, 3, 4, 5
PERM_ALGO_COMBINATORIC, PERM_ALGO_RYSER, PERM_ALGO_GLYNN, PERM_ALGO_GLYNN_ESYM, PERM_ALGO_AUTO, \
    PERM_ALGO_SWEEP = 0, 1, 2, 3, 4, 5
PERM_FLAG_WRAP = 0x1
PERM_FLAG_PAD_ONES = 0x2
PERM_BATCH_AUTOTUNE = 0x4
PERM_FLAG_SPARSE = 0x8
PERM_NOALLOC_SCRATCH_BYTES = 256 * 1024

_i32, _i64, _u32, _p, _d = ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p, \
    ctypes.c_double

_single = [_i32, _i32, _i32, _p, _i64, _i32, _p, _u32, _p]
for _name in ("perm_glynn", "perm_ryser", "perm_combinatoric", "perm_glynn_esym",
              "perm_glynn_noalloc", "perm_column_sweep"):
    getattr(lib, _name).argtypes = _single
    getattr(lib, _name).restype = _i32
lib.perm_auto.argtypes = _single + [_d, ctypes.POINTER(_i32)]
lib.perm_auto.restype = _i32
lib.perm_workspace_release.argtypes = []
lib.perm_workspace_release.restype = _i32
lib.perm_version.argtypes = []
lib.perm_version.restype = _i32
lib.perm_profile_enable.argtypes = [_i32]
lib.perm_profile_enable.restype = _i32
lib.perm_profile_last.argtypes = [ctypes.POINTER(_d)]
lib.perm_profile_last.restype = _i32
lib.perm_profile_durations.argtypes = [ctypes.POINTER(_d), _i32, ctypes.POINTER(_i32)]
lib.perm_profile_durations.restype = _i32
lib.perm_status_string.argtypes = [_i32]
lib.perm_status_string.restype = ctypes.c_char_p
lib.perm_batch_plan_create.argtypes = [_i32, _p, _p, _p, _p, _i32, _i32, _i32, _u32,
                                       ctypes.POINTER(_p)]
lib.perm_batch_plan_create.restype = _i32
lib.perm_batch_plan_run.argtypes = [_p, _p, _p, _p]
lib.perm_batch_plan_run.restype = _i32
lib.perm_batch_plan_destroy.argtypes = [_p]
lib.perm_gray_chunk.argtypes = [_i32, _i32, _i32, _i32, _p, _i64, _i32, _p, _u32, _i32, ctypes.c_uint64, _p]
lib.perm_gray_chunk.restype = _i32
lib.perm_batch_plan_packing.argtypes = [_p, _i32]
lib.perm_batch_plan_packing.restype = _i32
lib.perm_batch_plan_destroy.restype = _i32
for _name in ("perm_glynn_batched", "perm_ryser_batched", "perm_auto_batched"):
    getattr(lib, _name).argtypes = [_i32, _p, _p, _p, _p, _i32, _p, _i32, _p, _u32, _p]
    getattr(lib, _name).restype = _i32
lib.perm_selector_load.argtypes = [ctypes.c_char_p]
lib.perm_selector_load.restype = _i32
lib.perm_select.argtypes = [_i32, _i32, _i32, _d, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
lib.perm_select.restype = _i32
lib.perm_selector_features.argtypes = [_i32, _i32, _i32, _d, _p]
lib.perm_selector_features.restype = _i32
lib.perm_ryser_window_plan.argtypes = [_i32, _p, ctypes.c_uint64, _i32, ctypes.POINTER(_i32),
                                       ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                       ctypes.POINTER(ctypes.c_uint64), _p, _p, ctypes.c_uint64]
lib.perm_ryser_window_plan.restype = _i32
lib.perm_time.argtypes = [_i32, _i32, _i32, _i32, _p, _i64, _i32, _u32, _d, _i32, _p,
                          ctypes.POINTER(_d), ctypes.POINTER(_d)]
lib.perm_time.restype = _i32
_f = ctypes.c_float
lib.perm_mlp_forward.argtypes = [_p, _p, _p, _i32, _p, _p]
lib.perm_mlp_forward.restype = _i32
lib.perm_mlp_grad.argtypes = [_p, _p, _p, _p, _i32, _f, _p, _p, _p]
lib.perm_mlp_grad.restype = _i32
lib.perm_mlp_adam.argtypes = [_p, _p, _p, _f, _f, _f, _f, _i32, _p]
lib.perm_mlp_adam.restype = _i32
lib.perm_selector_train.argtypes = [_i32, _p, _p, _i32, _f, ctypes.c_uint64, _i32, _p, _p, _p,
                                    _p]
lib.perm_selector_train.restype = _i32
lib.perm_selector_save.argtypes = [ctypes.c_char_p, _p, _p, _p]
lib.perm_selector_save.restype = _i32
PERM_MLP_PARAMS = 4805


class PermError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = lib.perm_status_string(status).decode()
        super().__init__(f"{what}: {msg} (status {status})")


def check(status: int, what: str) -> None:
    if status != PERM_OK:
        raise PermError(status, what)
