"""ctypes declarations of the C ABI in include/wave2d.h (libwave2d.so)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwave2d.so")

OK, EINVAL, EUNSTABLE, ENOMEM, EDEVICE, EBUSY, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
P5, P9, P13, C9 = 5, 9, 13, 109
FIRST_CONVENTIONAL = 0x1
ALLOW_UNSTABLE = 0x2
PERIODIC = 0x4
KERNEL_SIMPLE = 0x100
F64, F32C = 0, 1
NOALLOC_MAX_BYTES = 64 << 20  # WAVE2D_NOALLOC_MAX_BYTES

I64 = ctypes.c_int64
D = ctypes.c_double
I = ctypes.c_int
U32 = ctypes.c_uint32
P = ctypes.c_void_p
SZ = ctypes.c_size_t


BATCH_GRAPH = 0x10000
BATCH_ROUNDS = 0x20000


class Tuning(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("rows", ctypes.c_int32)]


class Instance(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("h", ctypes.c_double), ("tau", ctypes.c_double), ("c", ctypes.c_double),
                ("scheme", ctypes.c_int32), ("flags", ctypes.c_uint32), ("steps", ctypes.c_int64),
                ("u0", ctypes.c_void_p), ("v0", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("lo", ctypes.c_void_p), ("d", ctypes.c_void_p)]


class BatchStats(ctypes.Structure):
    _fields_ = [("instances", ctypes.c_int64), ("rounds", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("lup", ctypes.c_int64), ("state_bytes", ctypes.c_int64), ("work_bytes", ctypes.c_int64),
                ("items", ctypes.c_int64), ("item_rows", ctypes.c_int64), ("persistent_items", ctypes.c_int64),
                ("stalled_waits", ctypes.c_int64), ("persistent_lup", ctypes.c_int64),
                ("persistent_bytes", ctypes.c_int64), ("last_persistent_ms", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("h", ctypes.c_double), ("tau", ctypes.c_double),
                ("c", ctypes.c_double), ("scheme", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("steps", ctypes.c_int64), ("nmodes", ctypes.c_int32), ("modes", ctypes.c_void_p),
                ("u0", ctypes.c_void_p), ("v0", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("u", ctypes.c_void_p), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("ld", ctypes.c_int64), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "admitted", "completed", "failed", "active", "queued",
                                              "quanta", "lup_done", "bytes_in_use", "bytes_budget")]


_SIGS = {
    "wave2d_lambda_max": (D, [I]),
    "wave2d_scheme_create": (I, [ctypes.c_int32, P, P, P]),
    "wave2d_weights": (I, [I, U32, D, P, P, P]),
    "wave2d_class_weights": (I, [I, U32, D, ctypes.c_int32, P, P, P]),
    "wave2d_status_str": (ctypes.c_char_p, [I]),
    "wave2d_last_error": (ctypes.c_char_p, []),
    "wave2d_work_bytes": (SZ, [I, I64, I64, I64]),
    "wave2d_first_step": (I, [I64, I64, I64, D, D, D, I, U32, P, P, P, P]),
    "wave2d_step": (I, [I64, I64, I64, D, D, D, I, U32, I64, P, P, P, SZ, P]),
    "wave2d_run": (I, [I64, I64, I64, D, D, D, I, U32, I64, P, P, P, P, P, SZ, P]),
    "wave2d_f32c_init": (I, [I64, I64, I64, P, P, P, P, P, P]),
    "wave2d_f32c_step": (I, [I64, I64, I64, D, D, D, I, U32, I64, P, P, P, P, SZ, P]),
    "wave2d_f32c_step_noalloc": (I, [I64, I64, I64, D, D, D, I, U32, I64, P, P, P, P]),
    "wave2d_f32c_export": (I, [I64, I64, I64, P, P, P, P]),
    "wave2d_f32c_run": (I, [I64, I64, I64, D, D, D, I, U32, I64, P, P, P, P, P, P, SZ, P]),
    "wave2d_norms": (I, [I64, I64, I64, P, P, P, P]),
    "wave2d_f32c_norms": (I, [I64, I64, I64, P, P, P, P, P]),
    "wave2d_set_tuning": (I, [I, I, P]),
    "wave2d_get_tuning": (I, [I, I, I64, I64, P]),
    "wave2d_release": (I, []),
    "wave2d_autotune": (I, [I, I, I64, I64, P, P]),
    "wave2d_batch_create": (I, [P, I64, U32, P]),
    "wave2d_batch_run": (I, [P, P]),
    "wave2d_batch_stats_get": (I, [P, P]),
    "wave2d_batch_autotune": (I, [P, P, P]),
    "wave2d_batch_set_rows_cap": (I, [P, ctypes.c_int32, P]),
    "wave2d_batch_destroy": (I, [P]),
    "wave2d_sine_series": (I, [I64, I64, I64, ctypes.c_int32, P, P, P, P]),
    "wave2d_server_create": (I, [SZ, U32, P]),
    "wave2d_server_submit": (I, [P, P, P]),
    "wave2d_server_poll": (I, [P, ctypes.c_uint64, P]),
    "wave2d_server_release": (I, [P, ctypes.c_uint64]),
    "wave2d_server_stats_get": (I, [P, P]),
    "wave2d_server_destroy": (I, [P]),
}

_lib = None


def exported_names():
    return list(_SIGS)


def load():
    """Load libwave2d.so.  Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class Wave2dError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{message} [{status}]")


def check(status: int) -> int:
    if status != OK:
        L = load()
        raise Wave2dError(status, f"{L.wave2d_status_str(status).decode()}: {L.wave2d_last_error().decode()}")
    return status
