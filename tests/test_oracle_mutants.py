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


# ---- the error-class rule ----------------------------------------------------------------

CLASS_MUTANTS = {
    "five-plus boundary at FC": ("if (c >= 0xF8) return 1;", "if (c >= 0xFC) return 1;"),
    "surrogate range short by one": ("cp <= 0xDFFF) return 6;", "cp < 0xDFFF) return 6;"),
    "three-byte overlong limit off by one": ("0x80, 0x800, 0x10000}", "0x80, 0x7FF, 0x10000}"),
    "too-large limit at 1FFFFF": ("if (cp > 0x10FFFF) return 5;", "if (cp > 0x1FFFFF) return 5;"),
    "last continuation unchecked": ("for (int k = 1; k < len; k++)\n        if (s + k >= n",
                                    "for (int k = 1; k < len - 1; k++)\n        if (s + k >= n"),
    "lead payload bit dropped": ("(c & (0x7F >> len))", "(c & (0x7F >> (len + 1)))"),
    "too large reported as surrogate": ("return 5;                               /* e)",
                                        "return 6;                               /* e)"),
}


def _class_pins_hold(lib):
    import itertools

    import test_oracle as to
    f = lib.oracle_first_error
    c = lib.oracle_error_class
    for b, off, cls, _ in to._golden_classes():
        if f(b, len(b)) != off or c(b, len(b), off) != cls:
            return False
    checks = [(to._encode(cp, 3), 6) for cp in range(0xD800, 0xE000, 31)] + [(to._encode(0xDFFF, 3), 6)]
    checks += [(to._encode(cp, 2), 4) for cp in range(0, 0x80, 5)]
    checks += [(to._encode(cp, 3), 4) for cp in range(0, 0x800, 37)] + [(to._encode(0x7FF, 3), 4)]
    checks += [(to._encode(cp, 4), 5) for cp in range(0x110000, 0x200000, 4099)]
    checks += [(to._encode(cp, 4), 0) for cp in (0x10000, 0x10FFFF)] + [(to._encode(0x800, 3), 0)]
    for b, cls in checks:
        s = f(b, len(b))
        if (c(b, len(b), s) if s >= 0 else 0) != cls:
            return False
    alpha = [0x00, 0x41, 0x80, 0xBF, 0xC0, 0xC2, 0xE0, 0xED, 0xF0, 0xF4, 0xF5, 0xF8, 0xFF, 0x90, 0xA0]
    for n in (1, 2, 3):
        for t in itertools.product(alpha, repeat=n):
            b = bytes(t)
            s = f(b, n)
            cls = c(b, n, s) if s >= 0 else 0
            try:
                b.decode("utf-8")
                ok = s == -1
            except UnicodeDecodeError as e:
                ok = e.start == s and cls != 0
                if e.reason == "unexpected end of data":
                    ok = ok and cls == 2
            if not ok:
                return False
    return True


def _build_classes(tmp_path, name, old, new):
    lib = _build(tmp_path, name, old, new)
    lib.oracle_error_class.restype = ctypes.c_int
    lib.oracle_error_class.argtypes = [ctypes.c_char_p, ctypes.c_int64, ctypes.c_int64]
    return lib


def test_unmutated_class_rule_passes(tmp_path):
    marker = "int oracle_error_class("
    assert _class_pins_hold(_build_classes(tmp_path, "same", marker, marker))


@pytest.mark.parametrize("name", sorted(CLASS_MUTANTS))
def test_class_mutant_is_caught(tmp_path, name):
    old, new = CLASS_MUTANTS[name]
    assert not _class_pins_hold(_build_classes(tmp_path, name, old, new)), f"pins missed mutant: {name}"


# ---- the batch form of the error-class rule -----------------------------------------------

CLASS_BATCH_MUTANTS = {
    "absolute offsets": ("oracle_error_class(data + st, len, first_err[k])",
                         "oracle_error_class(data, offsets[k + 1], first_err[k])"),
    "strings run to the batch end": ("int64_t st = offsets[k], len = offsets[k + 1] - st;",
                                     "int64_t st = offsets[k], len = offsets[n] - st;"),
    "offset zero taken as valid": ("first_err[k] < 0 ? 0", "first_err[k] <= 0 ? 0"),
}


def _class_batch_pins_hold(lib):
    import test_oracle as to
    data, offsets, ferr, cls = to._golden_class_batch()
    out = np.zeros(cls.size, np.uint8)
    lib.oracle_error_class_batch(data.ctypes.data, offsets.ctypes.data, cls.size, ferr.ctypes.data,
                                 out.ctypes.data)
    return out.tolist() == cls.tolist()


def _build_class_batch(tmp_path, name, old, new):
    lib = _build(tmp_path, name, old, new)
    lib.oracle_error_class_batch.restype = ctypes.c_int
    lib.oracle_error_class_batch.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_void_p]
    return lib


def test_unmutated_class_batch_passes(tmp_path):
    marker = "int oracle_error_class_batch("
    assert _class_batch_pins_hold(_build_class_batch(tmp_path, "same", marker, marker))


@pytest.mark.parametrize("name", sorted(CLASS_BATCH_MUTANTS))
def test_class_batch_mutant_is_caught(tmp_path, name):
    old, new = CLASS_BATCH_MUTANTS[name]
    assert not _class_batch_pins_hold(_build_class_batch(tmp_path, name, old, new)), f"pins missed mutant: {name}"
