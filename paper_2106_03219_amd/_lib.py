"""ctypes declarations of libomprt.so (the C ABI in include/omprt.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation of any entry point.
"""
from __future__ import annotations

import atexit
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libomprt.so")

OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_NOMEM, ERR_DEVICE = range(5)
I32, I64, F32, F64, BF16 = range(5)
SUM, MAX, MIN, PROD, BAND, BOR, BXOR, LAND, LOR = range(9)
ATOMIC_ADD, ATOMIC_INC, ATOMIC_MAX, ATOMIC_EXCHANGE, ATOMIC_CAS = range(5)
CFG_NO_MODEL = 0x1
CFG_STATIC_TILES = 0x2
CFG_HIST_TEAM_COPY = 0x4
CFG_HIST_DIRECT = 0x8
CFG_EXACT_THREAD_MAP = 0x10
CFG_HIST_PARTITION = 0x20
CFG_HIST_RANGES = 0x40
CFG_HIST_TILE_SORT = 0x80


class Sched(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("num_teams", ctypes.c_int32),
                ("threads_per_team", ctypes.c_int32), ("dist_chunk", ctypes.c_int64),
                ("chunk", ctypes.c_int64)]


class Config(ctypes.Structure):
    _fields_ = [("num_teams", ctypes.c_int32), ("threads_per_team", ctypes.c_int32),
                ("vec_bytes", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("tile_kib", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Segment(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_void_p), ("n", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("op", ctypes.c_int32), ("d_x", ctypes.c_void_p)]


class UdrSource(ctypes.Structure):
    _fields_ = [("type_def", ctypes.c_char_p), ("initializer", ctypes.c_char_p),
                ("combiner", ctypes.c_char_p), ("body", ctypes.c_char_p),
                ("acc_bytes", ctypes.c_int32)]


class MlpDims(ctypes.Structure):
    _fields_ = [("F", ctypes.c_int32), ("H1", ctypes.c_int32), ("H2", ctypes.c_int32),
                ("K", ctypes.c_int32)]


# name -> (restype, argtypes); every symbol declared in include/omprt.h
_i32, _i64, _u32, _f32, _p = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_float, ctypes.c_void_p
_S, _C, _D = ctypes.POINTER(Sched), ctypes.POINTER(Config), ctypes.POINTER(MlpDims)
SIGNATURES = {
    "omprt_for_static_bounds": (_i32, [_S, _i32, _i32, _i64, ctypes.POINTER(_i64),
                                       ctypes.POINTER(_i64), ctypes.POINTER(_i32)]),
    "omprt_sched_count": (_i32, [_S, _i32, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "omprt_static_map": (_i32, [_S, _p, _p, _p]),
    "omprt_reduce": (_i32, [_p, _i64, _i32, _i32, _p, _C, _p]),
    "omprt_reduce_noalloc": (_i32, [_p, _i64, _i32, _i32, _p, _C, _p]),
    "omprt_reduce_array": (_i32, [_p, _i64, _i64, _i32, _i32, _p, _C, _p]),
    "omprt_reduce_loc": (_i32, [_p, _i64, _i32, _i32, _p, _p, _C, _p]),
    "omprt_reduce_multi": (_i32, [_p, _i64, _i32, _i32, _p, _p, _C, _p]),
    "omprt_histogram": (_i32, [_p, _i64, _i32, _p, _C, _p]),
    "omprt_udr_declare": (_i32, [ctypes.POINTER(UdrSource), _i32, ctypes.POINTER(_i32)]),
    "omprt_reduce_udr": (_i32, [_i32, _p, _i64, _p, _C, _p]),
    "omprt_generic_power": (_i32, [_p, _p, _i64, _i32, _i32, _i32, _p, _p]),
    "omprt_reduce_array_plan": (_i32, [_i64, _i64, _i32, _i32, _i32, _C, _p]),
    "omprt_reduce_batched": (_i32, [ctypes.POINTER(Segment), _i32, _C, _p]),
    "omprt_reduce_each": (_i32, [ctypes.POINTER(Segment), _i32, _C, _p]),
    "omprt_axpy_sum": (_i32, [_f32, _p, _p, _p, _S, _C, _p]),
    "omprt_region_axpy_sum": (_i32, [_f32, _p, _p, _p, _S, _i64, _i32, _C, _p]),
    "omprt_empty_region": (_i32, [_S, _p, _p]),
    "omprt_atomic_apply": (_i32, [_i32, _p, _i64, _p, _p, _p, _p, _i64, _p]),
    "omprt_queue_chunk": (_i32, [_i32, _i64, _i32, _i64, _i64, _p, _p]),
    "omprt_queue_map": (_i32, [_S, _i32, _i32, _p, _p, _p, _p]),
    "omprt_axpy_sum_queue": (_i32, [ctypes.c_float, _p, _p, _p, _S, _i32, _p]),
    "omprt_mlp_param_count": (_i64, [_D]),
    "omprt_mlp_forward": (_i32, [_D, _p, _p, _i32, _p, _p]),
    "omprt_mlp_loss_grad": (_i32, [_D, _p, _p, _p, _i32, _p, _p, _p]),
    "omprt_mlp_adam": (_i32, [_p, _p, _p, _p, _i64, _i32, _f32, _f32, _f32, _f32, _p]),
    "omprt_mlp_adam_counted": (_i32, [_p, _p, _p, _p, _i64, _p, _f32, _f32, _f32, _f32, _p]),
    "omprt_model_load": (_i32, [ctypes.c_char_p]),
    "omprt_model_features": (_i32, [_i64, _i32, _i32, _i32, _i64, ctypes.POINTER(_f32)]),
    "omprt_resolve_config": (_i32, [_i64, _i32, _i32, _i32, _i64, _C, _C, ctypes.POINTER(_i32)]),
    "omprt_tune_set": (_i32, [_i32, _i32, _i32, _i32, _C]),
    "omprt_workspace_reserve": (_i32, [_p, _i32, _i32]),
    "omprt_workspace_reset": (_i32, [_p]),
    "omprt_workspace_status": (_i32, [_p, ctypes.POINTER(_i32)]),
    "omprt_last_error": (ctypes.c_char_p, []),
    "omprt_version": (ctypes.c_char_p, []),
    "omprt_finalize": (_i32, []),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libomprt.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2106_03219_amd.build` "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    # explicit teardown while the HIP runtime is still up: the library frees its
    # device memory here, never from static destructors at process exit
    atexit.register(_finalize_at_exit)
    return lib


def _finalize_at_exit() -> None:
    if _lib is not None:
        try:
            _lib.omprt_finalize()
        except Exception:   # noqa: BLE001 -- nothing can be reported at exit
            pass


class OmprtError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != OK:
        msg = load().omprt_last_error().decode(errors="replace")
        raise OmprtError(status, where, msg)
