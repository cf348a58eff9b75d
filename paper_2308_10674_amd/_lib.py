"""ctypes declarations of libptyc.so (the C ABI in include/ptyc.h)."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libptyc.so")

PTYC_OK = 0
PTYC_ERR_ARG = -1
PTYC_ERR_BOUNDS = -2
PTYC_ERR_OOM = -3
PTYC_ERR_HIP = -4
PTYC_ERR_STATE = -5
PTYC_MEM_HOST = 0
PTYC_MEM_DEVICE = 1
PTYC_MODE_STRICT = 0
PTYC_MODE_COLOURED = 1
PTYC_FORM_DEFAULT = 0
PTYC_FORM_BATCH = 1
PTYC_FORM_PERSISTENT = 2
PTYC_FORM_GRAPH = 3
PTYC_TILE_MAX = 8
PTYC_NOALLOC_BYTES = 32 << 20
PTYC_MULTI_VARIANTS = 8
PTYC_KERNEL_ROWS_FWD = 0
PTYC_KERNEL_COLS = 1
PTYC_KERNEL_ROWS_INV = 2
PTYC_KERNEL_SWEEP = 3
PTYC_KERNEL_GRAPH = 4
PTYC_KERNEL_STRICT = 5
KERNEL_NAMES = {0: "k_rows_fwd", 1: "k_cols", 2: "k_rows_inv", 3: "k_sweep", 4: "sweep_graph", 5: "k_strict"}
PTYC_I_IS_SQRT = 1
PTYC_I_CENTERED = 2

STATUS_NAMES = {
    PTYC_ERR_ARG: "PTYC_ERR_ARG", PTYC_ERR_BOUNDS: "PTYC_ERR_BOUNDS", PTYC_ERR_OOM: "PTYC_ERR_OOM",
    PTYC_ERR_HIP: "PTYC_ERR_HIP", PTYC_ERR_STATE: "PTYC_ERR_STATE",
}


class Config(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("h", C.c_int32), ("w", C.c_int32),
        ("alpha", C.c_float), ("beta", C.c_float),
        ("mode", C.c_int32), ("max_batch", C.c_int32),
        ("seed", C.c_uint64), ("flags", C.c_uint32), ("reserved", C.c_int32),
    ]


class Ingest(C.Structure):
    _fields_ = [
        ("frame_h", C.c_int32), ("frame_w", C.c_int32), ("crop_y", C.c_int32), ("crop_x", C.c_int32),
        ("orient", C.c_int32), ("scale", C.c_float), ("flags", C.c_uint32), ("reserved", C.c_int32),
    ]


_P = C.c_void_p
_I64P = C.POINTER(C.c_int64)
_I32P = C.POINTER(C.c_int32)
_DP = C.POINTER(C.c_double)

SIGNATURES = {
    "ptyc_init": (C.c_int, [C.POINTER(_P), C.POINTER(Config), _P, _P, C.c_int, _P]),
    "ptyc_add_positions": (C.c_int, [_P, C.c_int64, _P, _P, C.c_int]),
    "ptyc_sweep": (C.c_int, [_P, C.c_int32, _I64P, C.c_int64, _I64P, C.c_int64, _DP]),
    "ptyc_sweep_noalloc": (C.c_int, [_P, C.c_int32, _I64P, C.c_int64, _I64P, C.c_int64, _DP]),
    "ptyc_sweep_multi": (C.c_int, [C.POINTER(_P), C.c_int32, C.c_int32, _DP]),
    "ptyc_average": (C.c_int, [C.POINTER(_P), C.c_int32]),
    "ptyc_multi_variant_count": (C.c_int, []),
    "ptyc_set_multi_variant": (C.c_int, [_P, C.c_int]),
    "ptyc_get_multi_variant": (C.c_int, [_P]),
    "ptyc_tune_multi": (C.c_int, [C.POINTER(_P), C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "ptyc_get_schedule": (C.c_int, [_P, _I64P, _I64P, _I64P]),
    "ptyc_set_ingest": (C.c_int, [_P, C.POINTER(Ingest)]),
    "ptyc_set_mask": (C.c_int, [_P, _P, C.c_int]),
    "ptyc_get_patterns": (C.c_int, [_P, C.c_int64, C.c_int64, _P, C.c_int]),
    "ptyc_get_object": (C.c_int, [_P, _P, C.c_int]),
    "ptyc_get_probe": (C.c_int, [_P, _P, C.c_int]),
    "ptyc_set_object": (C.c_int, [_P, _P, C.c_int]),
    "ptyc_set_probe": (C.c_int, [_P, _P, C.c_int]),
    "ptyc_amp_loss": (C.c_int, [_P, _P, _P, _I64P, C.c_int64, C.c_float, _P, _P, _DP]),
    "ptyc_amp_loss_async": (C.c_int, [_P, _P, _P, _I64P, C.c_int64, _P, _P, _P]),
    "ptyc_scale_c64": (C.c_int, [_P, _P, C.c_int64, _P]),
    "ptyc_set_form": (C.c_int, [_P, C.c_int]),
    "ptyc_profile": (C.c_int, [_P, C.c_int]),
    "ptyc_profile_read": (C.c_int, [_P, C.c_int, _DP, _I64P, _I64P]),
    "ptyc_get_form": (C.c_int, [_P]),
    "ptyc_tile_count": (C.c_int, [_P]),
    "ptyc_set_tile": (C.c_int, [_P, C.c_int]),
    "ptyc_get_tile": (C.c_int, [_P]),
    "ptyc_tune": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "ptyc_num_positions": (C.c_int64, [_P]),
    "ptyc_sweep_count": (C.c_int64, [_P]),
    "ptyc_synchronize": (C.c_int, [_P]),
    "ptyc_destroy": (None, [_P]),
    "ptyc_last_error": (C.c_char_p, [_P]),
    "ptyc_init_error": (C.c_char_p, []),
    "ptyc_colour": (C.c_int, [C.c_int64, _P, C.c_int32, C.c_int32, _I32P, _I32P]),
    "ptyc_check_batches": (C.c_int, [C.c_int64, _P, C.c_int32, _I64P, C.c_int64, _I64P, C.c_int64]),
    "ptyc_version": (C.c_int, []),
}

_lib = None


def lib() -> C.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2308_10674_amd.build.build() "
                              "(there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class PtycError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
