"""CPU baselines for measurements (never used by the library's validation path).

``host_lookup`` is the section 6 lookup algorithm with AVX2 on the host, the
way the paper runs it: a stronger CPU reference point than the branchy oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "host_lookup.c")
_LIB = os.path.join(_HERE, "libhost_lookup.so")
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-shared", "-fPIC", "-pthread", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.host_lookup_validate.restype = ctypes.c_int
        lib.host_lookup_validate.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        lib.host_lookup_validate_mt.restype = ctypes.c_int
        lib.host_lookup_validate_mt.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
        lib.host_lookup_supported.restype = ctypes.c_int
        _lib = lib
    return _lib


def supported() -> bool:
    return bool(_load().host_lookup_supported())


def is_valid(buf: np.ndarray, nthreads: int = 1) -> bool:
    a = np.ascontiguousarray(buf, dtype=np.uint8)
    lib = _load()
    r = lib.host_lookup_validate_mt(a.ctypes.data if a.size else None, a.size, nthreads) if nthreads > 1 else \
        lib.host_lookup_validate(a.ctypes.data if a.size else None, a.size)
    if r < 0:
        raise RuntimeError("host CPU lacks AVX2")
    return bool(r)
