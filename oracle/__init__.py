"""UTF-8 validation oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU product path never does: it has
no fallback to the CPU.

Two independent references live here:

* ``first_error`` / ``first_error_batch`` -- the plain branchy range walk of
  Algorithm 1 (section 4) over the byte ranges of Table 1 (section 2), written
  in C (``utf8_oracle.c``).  It returns the first-error offset: the length of
  the longest valid prefix made of whole characters, or -1 for valid input.
* ``error_class`` / ``error_class_batch`` -- which of the six rules of section 3
  (a..f, coded 1..6) the first ill-formed character breaks: malformed rules
  first (5+ byte, too long, too short), then overlong / too large / surrogate
  on the decoded code point.
* ``lookup_model`` -- the paper's lookup algorithm (section 6) written out step
  by step in numpy, with its three nibble tables derived from the error
  patterns of Table 8.  It is pinned to the worked example of Table 9.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "utf8_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle_utf8.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc into ``oracle/liboracle_utf8.so``."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-shared", "-fPIC", "-pthread",
                               "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.oracle_first_error.restype = ctypes.c_int64
        lib.oracle_first_error.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        lib.oracle_first_error_batch.restype = ctypes.c_int
        lib.oracle_first_error_batch.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.oracle_error_class.restype = ctypes.c_int
        lib.oracle_error_class.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64]
        lib.oracle_error_class_batch.restype = ctypes.c_int
        lib.oracle_error_class_batch.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                 ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_exhaustive_hist.restype = ctypes.c_int
        lib.oracle_exhaustive_hist.argtypes = [ctypes.c_int, ctypes.c_void_p]
        _lib = lib
    return _lib


def _as_u8(buf) -> np.ndarray:
    if isinstance(buf, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(buf), dtype=np.uint8)
    a = np.ascontiguousarray(buf)
    if a.dtype != np.uint8:
        raise TypeError("oracle input must be uint8")
    return a.reshape(-1)


def first_error(buf) -> int:
    """First-error offset of one byte string (-1 if it is valid UTF-8)."""
    a = _as_u8(buf)
    return int(_load().oracle_first_error(a.ctypes.data if a.size else None, a.size))


ERROR_CLASSES = {0: "valid", 1: "five_plus_byte", 2: "too_short", 3: "too_long", 4: "overlong",
                 5: "too_large", 6: "surrogate"}


def error_class(buf, first_err: int | None = None) -> int:
    """Section 3 rule (1..6 = a..f) broken by the first ill-formed character, 0 if valid."""
    a = _as_u8(buf)
    s = first_error(a) if first_err is None else int(first_err)
    return int(_load().oracle_error_class(a.ctypes.data if a.size else None, a.size, s))


def error_class_batch(data, offsets, first_err) -> np.ndarray:
    d = _as_u8(data)
    o = np.ascontiguousarray(offsets, dtype=np.int64)
    f = np.ascontiguousarray(first_err, dtype=np.int64)
    out = np.zeros(o.size - 1, dtype=np.uint8)
    if _load().oracle_error_class_batch(d.ctypes.data if d.size else None, o.ctypes.data, o.size - 1,
                                        f.ctypes.data, out.ctypes.data):
        raise ValueError("bad batch")
    return out


def is_valid(buf) -> bool:
    return first_error(buf) < 0


def first_error_batch(data, offsets, nthreads: int | None = None):
    """Per-string (flags uint8, first_err int64) for string k = data[offsets[k]:offsets[k+1]].

    Offsets in ``first_err`` are relative to each string's start.
    """
    d = _as_u8(data)
    off = np.ascontiguousarray(offsets, dtype=np.int64).reshape(-1)
    n = off.size - 1
    if n < 0:
        raise ValueError("offsets must hold n+1 entries")
    if n and (off[0] < 0 or off[-1] > d.size or np.any(np.diff(off) < 0)):
        raise ValueError("offsets must be non-decreasing and inside data")
    flags = np.empty(n, dtype=np.uint8)
    ferr = np.empty(n, dtype=np.int64)
    if n == 0:
        return flags, ferr
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    rc = _load().oracle_first_error_batch(d.ctypes.data if d.size else None, off.ctypes.data, n,
                                          flags.ctypes.data, ferr.ctypes.data, int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle batch failed ({rc})")
    return flags, ferr


def exhaustive_hist(length: int) -> np.ndarray:
    """Counts over all 256**length strings: [k] = #first_err == k (k < length), [length] = #valid."""
    hist = np.zeros(length + 1, dtype=np.uint64)
    if _load().oracle_exhaustive_hist(int(length), hist.ctypes.data) != 0:
        raise ValueError("length must be in 0..4")
    return hist
