"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a temporary copy of the oracle's C source (a
wrong range bound, a dropped check, an off-by-one), builds it with gcc, and
checks that at least one pin fails: the closed-form histogram of all strings of
length <= 3, the paper's labelled vectors, or CPython's decoder on the boundary
alphabet of length 4.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from conftest import read_labelled_vectors
from test_oracle import BOUNDARY_ALPHABET, _cpython_first_error, bad_start_count, valid_count

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "utf8_oracle.c")

MUTANTS = {
    "E0 overlong accepted": ("lo1 = 0xA0;", "lo1 = 0x80;"),
    "ED surrogates accepted": ("{ len = 3; hi1 = 0x9F; }", "{ len = 3; hi1 = 0xBF; }"),
    "F0 overlong accepted": ("lo1 = 0x90;", "lo1 = 0x80;"),
    "F4 as printed in Algorithm 1": ("{ len = 4; hi1 = 0x8F; }", "{ len = 4; hi1 = 0x9F; }"),
    "C0/C1 accepted": ("in_range(c, 0xC2, 0xDF)", "in_range(c, 0xC0, 0xDF)"),
    "F5..F7 accepted": ("in_range(c, 0xF1, 0xF3)", "in_range(c, 0xF1, 0xF7)"),
    "too-short check off by one": ("if (i + len > n) return 0;", "if (i + len > n + 1) return 0;"),
    "last continuation unchecked": ("for (int k = 2; k < len; k++)", "for (int k = 2; k < len - 1; k++)"),
    "continuation range too wide": ("uint8_t lo1 = 0x80, hi1 = 0xBF;", "uint8_t lo1 = 0x80, hi1 = 0xC0;"),
    "offset off by one": ("if (len == 0) return i;", "if (len == 0) return i + (i > 0);"),
    "three-byte leads EE..EF dropped": ("|| in_range(c, 0xEE, 0xEF)", "|| in_range(c, 0xEE, 0xEE)"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "mutant.so"
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-pthread", "-o", str(so), str(path)])
    lib = ctypes.CDLL(str(so))
    lib.oracle_first_error.restype = ctypes.c_int64
    lib.oracle_first_error.argtypes = [ctypes.c_char_p, ctypes.c_int64]
    lib.oracle_exhaustive_hist.argtypes = [ctypes.c_int, ctypes.c_void_p]
    return lib


def _pins_hold(lib):
    for n in range(4):
        hist = np.zeros(n + 1, np.uint64)
        lib.oracle_exhaustive_hist(n, hist.ctypes.data)
        if hist.tolist() != [valid_count(k) * bad_start_count(n - k) for k in range(n)] + [valid_count(n)]:
            return False
    for b, exp, _, _ in read_labelled_vectors():
        if lib.oracle_first_error(b, len(b)) != exp:
            return False
    alpha = np.frombuffer(BOUNDARY_ALPHABET, np.uint8)
    idx = np.indices((alpha.size,) * 4).reshape(4, -1).T
    for s in alpha[idx]:
        b = bytes(s)
        if lib.oracle_first_error(b, 4) != _cpython_first_error(b):
            return False
    idx = np.indices((alpha.size,) * 3).reshape(3, -1).T
    for s in alpha[idx]:
        b = bytes(s)
        for n in (1, 2, 3):  # memory after the n bytes holds continuation bytes
            if lib.oracle_first_error(b[:n] + b"\x80\xbf\x80", n) != _cpython_first_error(b[:n]):
                return False
    return True


def test_unmutated_oracle_passes(tmp_path):
    src = open(SRC).read()
    (tmp_path / "same.c").write_text(src)
    so = tmp_path / "same.so"
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-pthread", "-o", str(so), str(tmp_path / "same.c")])
    lib = ctypes.CDLL(str(so))
    lib.oracle_first_error.restype = ctypes.c_int64
    lib.oracle_first_error.argtypes = [ctypes.c_char_p, ctypes.c_int64]
    lib.oracle_exhaustive_hist.argtypes = [ctypes.c_int, ctypes.c_void_p]
    assert _pins_hold(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    assert not _pins_hold(_build(tmp_path, name, old, new)), f"pins missed mutant: {name}"
