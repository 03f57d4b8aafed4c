"""ctypes binding of libutf8v.so (argument marshalling only).

Every function here calls the C-ABI declared in include/utf8v.h; all validation
work runs in the library's HIP kernels.  There is no CPU fallback: loading
fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libutf8v.so")

UTF8V_OK = 0
UTF8V_EINVAL = -1
UTF8V_ENOTDEVICE = -2
UTF8V_EHIP = -3
UTF8V_ENOMEM = -4

# Every function the header exports, with its ctypes signature.
_i32, _i64, _sz, _vp = ctypes.c_int, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p


class Config(ctypes.Structure):
    _fields_ = [("unroll", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32), ("ascii", ctypes.c_int32),
                ("batch_waves_per_cu", ctypes.c_int32), ("batch_ascii", ctypes.c_int32),
                ("batch_unroll", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class ServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("max_batch_bytes", ctypes.c_uint64),
                ("max_batch_strings", ctypes.c_int64), ("max_batch_requests", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("streams", ctypes.c_int32), ("max_pending", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


_u64 = ctypes.c_uint64
_pcfg = ctypes.POINTER(ServerConfig)

SIGNATURES = {
    "utf8_validate": (ctypes.c_bool, [_vp, _sz]),
    "utf8v_validate_ex": (_i32, [_vp, _sz, _vp, _vp]),
    "utf8v_validate_async": (_i32, [_vp, _sz, _vp, _vp]),
    "utf8_validate_batch": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "utf8v_validate_batch_async": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp]),
    "utf8v_validate_batch_graph": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp]),
    "utf8v_validate_batch_noalloc": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp]),
    "utf8v_check_offsets": (_i32, [_vp, _i64, _vp]),
    "utf8v_get_config": (_i32, [ctypes.POINTER(Config)]),
    "utf8v_set_config": (_i32, [ctypes.POINTER(Config)]),
    "utf8v_classify": (_i32, [_vp, _sz, _vp, _vp, _vp]),
    "utf8v_read_ceiling": (_i32, [_vp, _sz, _vp, _vp]),
    "utf8v_copy": (_i32, [_vp, _vp, _sz, _vp]),
    "utf8v_last_status": (_i32, []),
    "utf8v_strerror": (ctypes.c_char_p, [_i32]),
    "utf8v_last_hip_error": (_i32, []),
    "utf8v_num_cus": (_i32, []),
    "utf8v_release": (_i32, []),
    "utf8v_server_default_config": (_i32, [_pcfg]),
    "utf8v_server_create": (_i32, [_pcfg, ctypes.POINTER(_vp)]),
    "utf8v_server_submit": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, ctypes.POINTER(_u64)]),
    "utf8v_server_poll": (_i32, [_vp, _u64, ctypes.POINTER(_i64)]),
    "utf8v_server_wait": (_i32, [_vp, _u64, ctypes.POINTER(_i64)]),
    "utf8v_server_stats": (_i32, [_vp, _vp]),
    "utf8v_server_destroy": (_i32, [_vp]),
    "utf8v_clock_ns": (_i64, []),
    "utf8v_copy_validate": (_i32, [_vp, _vp, _sz, _vp, _vp]),
    "utf8v_error_class": (_i32, [_vp, _sz, _vp, _vp, _vp]),
    "utf8v_error_classes": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp]),
    "utf8v_stream_create": (_i32, [ctypes.POINTER(_vp), _vp]),
    "utf8v_stream_update": (_i32, [_vp, _vp, _sz, _vp]),
    "utf8v_stream_finish": (_i32, [_vp, ctypes.POINTER(_i64), _vp]),
    "utf8v_stream_reset": (_i32, [_vp, _vp]),
    "utf8v_stream_position": (_i64, [_vp]),
    "utf8v_stream_destroy": (_i32, [_vp]),
    "utf8v_autotune_single": (_i32, [_vp, _vp, _i32, _i32, ctypes.POINTER(Config), _vp, _i32]),
    "utf8v_autotune_batch": (_i32, [_vp, _vp, _i64, _vp, _vp, _i32, ctypes.POINTER(Config), _vp, _i32]),
    "utf8v_serve_replay": (_i32, [_pcfg, _i32, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _i64, _vp, _vp]),
}

_lib = None


class Utf8vError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        msg = lib.utf8v_strerror(status).decode()
        if status == UTF8V_EHIP:
            msg += f" (hipError {lib.utf8v_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{status}]")
        self.status = status


def load():
    """Load libutf8v.so (built by paper_2010_03090_amd.build); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2010_03090_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int, where: str) -> int:
    if status < 0:
        raise Utf8vError(status, where)
    return status
