"""Seeded synthetic workloads for UTF-8 validation (generation only, no validation).

The C core (``synth.c``) encodes code points drawn from a per-variant mix of
UTF-8 byte lengths, injects single errors whose first-error offset is known by
construction, and lays out CSR string batches.  Tests, the benchmark and the
serving load generator all draw their inputs from here; the oracle and the GPU
validator both consume them and neither is used to make them.

Workload shapes (the paper's inputs are not available; these stand in):

* ``mixed``: code points 50% U+0000-007F, 20% U+0080-07FF, 20% U+0800-FFFF
  (no surrogates), 10% U+10000-10FFFF.
* ``ascii``, ``latin`` (85% 1-byte / 15% 2-byte), ``cjk`` (10% / 90% 3-byte),
  ``emoji`` (40% / 60% 4-byte), ``random`` (uniform bytes, almost surely invalid).
* ``unif1`` .. ``unif4``: the paper's randomized inputs (section 7.3), the byte
  length of each code point uniform over {1}, {1,2}, {1,2,3} or {1,2,3,4}.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

VARIANTS = {"ascii": 0, "latin": 1, "cjk": 2, "emoji": 3, "random": 4, "mixed": 5,
            "unif1": 6, "unif2": 7, "unif3": 8, "unif4": 9}
ERROR_CLASSES = {"lone_continuation": 0, "truncated_lead": 1, "overlong": 2, "too_large": 3,
                 "surrogate": 4, "five_plus_lead": 5, "cut_at_end": 6}


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-shared", "-fPIC", "-pthread", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        i64, vp, ci, u64 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64
        lib.synth_text.argtypes = [vp, i64, ci, u64, ci]
        lib.synth_text.restype = ci
        lib.synth_inject.argtypes = [vp, i64, i64, ci, u64]
        lib.synth_inject.restype = i64
        lib.synth_lengths.argtypes = [vp, i64, ci, ctypes.c_double, ctypes.c_double, i64, i64, u64]
        lib.synth_lengths.restype = ci
        lib.synth_batch_text.argtypes = [vp, vp, vp, i64, u64, ci]
        lib.synth_batch_text.restype = ci
        _lib = lib
    return _lib


def _threads(n):
    return int(n) if n else min(16, os.cpu_count() or 1)


def _mix(seed: int, *salt: int) -> int:
    h = (int(seed) * 0x9E3779B97F4A7C15 + 0x2545F4914F6CDD1D) & (2**64 - 1)
    for s in salt:
        h ^= (int(s) + 0x9E3779B97F4A7C15 + (h << 6) + (h >> 2)) & (2**64 - 1)
    return h & (2**64 - 1)


def text(n: int, variant: str = "mixed", seed: int = 0, nthreads: int | None = None) -> np.ndarray:
    """Exactly n bytes of valid text of the variant (or random bytes)."""
    out = np.empty(int(n), dtype=np.uint8)
    rc = _load().synth_text(out.ctypes.data if n else None, int(n), VARIANTS[variant], _mix(seed, 1),
                            _threads(nthreads))
    if rc:
        raise ValueError("synth_text failed")
    return out


def inject(buf: np.ndarray, pos: int, cls: int | str, seed: int) -> int:
    """Inject one error at the first character boundary >= pos (in place); returns its offset."""
    if isinstance(cls, str):
        cls = ERROR_CLASSES[cls]
    if buf.dtype != np.uint8 or not buf.flags.c_contiguous:
        raise TypeError("buf must be a contiguous uint8 array")
    return int(_load().synth_inject(buf.ctypes.data, buf.size, int(pos), int(cls), _mix(seed, 2)))


def inject_random(buf: np.ndarray, seed: int, lo: int = 0, hi: int | None = None, cls=None) -> tuple[int, int]:
    """One error of a random class (uniform over the seven) at a uniform offset in [lo, hi)."""
    rng = np.random.default_rng(_mix(seed, 3))
    hi = buf.size if hi is None else hi
    for _ in range(64):
        c = int(rng.integers(0, len(ERROR_CLASSES))) if cls is None else int(cls)
        pos = int(rng.integers(lo, max(lo + 1, hi)))
        s = inject(buf, pos, c, int(rng.integers(0, 2**62)))
        if s >= 0:
            return s, c
    raise RuntimeError("could not inject an error")


def lengths(n: int, dist: str, a: float, b: float, lo: int, hi: int, seed: int) -> np.ndarray:
    """String lengths: lognormal(median a, sigma b) or Pareto(x_m a, alpha b), clipped to [lo, hi]."""
    out = np.empty(int(n), dtype=np.int64)
    d = {"lognormal": 0, "pareto": 1}[dist]
    if _load().synth_lengths(out.ctypes.data if n else None, int(n), d, float(a), float(b), int(lo), int(hi),
                             _mix(seed, 4)):
        raise ValueError("synth_lengths failed")
    return out


def batch_from_lengths(lens: np.ndarray, variants, seed: int, err_frac: float = 0.0, base: int = 0,
                       nthreads: int | None = None):
    """CSR batch with the given string lengths.

    ``variants`` is a variant name or one name per string.  A fraction
    ``err_frac`` of the strings (chosen at random) get one injected error.
    Returns (data uint8, offsets int64[n+1], expected first_err int64[n]);
    ``offsets[0] == base`` (leading bytes before it are random filler).
    """
    lens = np.ascontiguousarray(lens, dtype=np.int64)
    n = lens.size
    offsets = np.empty(n + 1, dtype=np.int64)
    offsets[0] = base
    np.cumsum(lens, out=offsets[1:])
    offsets[1:] += base
    data = np.empty(int(offsets[-1]), dtype=np.uint8)
    if base:
        data[:base] = np.frombuffer(np.random.default_rng(seed).bytes(base), np.uint8)
    if isinstance(variants, str):
        var = np.full(n, VARIANTS[variants], dtype=np.int32)
    else:
        var = np.array([VARIANTS[v] if isinstance(v, str) else int(v) for v in variants], dtype=np.int32)
    if n and _load().synth_batch_text(data.ctypes.data, offsets.ctypes.data, var.ctypes.data, n,
                                      _mix(seed, 5), _threads(nthreads)):
        raise ValueError("synth_batch_text failed")
    expected = np.full(n, -1, dtype=np.int64)
    if err_frac > 0 and n:
        rng = np.random.default_rng(_mix(seed, 6))
        k_err = int(round(err_frac * n))
        chosen = np.sort(rng.choice(n, size=k_err, replace=False)) if k_err else np.zeros(0, np.int64)
        for k in chosen:
            s0, e0 = int(offsets[k]), int(offsets[k + 1])
            view = data[s0:e0]
            if view.size == 0:
                continue
            s, _ = inject_random(view, int(rng.integers(0, 2**62)))
            expected[k] = s
    return data, offsets, expected


# ---- named workloads --------------------------------------------------------------------

def single_buffer_with_errors(n: int, variant: str, seed: int, copies: int):
    """A valid buffer and `copies` corrupted copies, each with one random error at a uniform offset.

    Returns (clean, [(corrupted, expected_first_err, class), ...]).
    """
    clean = text(n, variant, seed)
    out = []
    rng = np.random.default_rng(_mix(seed, 7))
    for c in range(copies):
        buf = clean.copy()
        s, cls = inject_random(buf, int(rng.integers(0, 2**62)))
        out.append((buf, s, cls))
    return clean, out


def tail_error_copy(clean: np.ndarray, seed: int):
    """A copy of valid text with one error whose first-error offset lies in the last 4 bytes."""
    buf = clean.copy()
    n = buf.size
    rng = np.random.default_rng(_mix(seed, 8))
    for _ in range(64):
        cls = int(rng.integers(0, len(ERROR_CLASSES)))
        tmp = buf[max(0, n - 16):].copy()
        s = inject(tmp, max(0, tmp.size - 4), cls, int(rng.integers(0, 2**62)))
        if s >= 0 and s >= tmp.size - 4:
            buf[max(0, n - 16):] = tmp
            return buf, s + max(0, n - 16), cls
    raise RuntimeError("no tail error fitted")


def lognormal_batch(n_strings: int, seed: int, variant: str = "mixed", err_frac: float = 0.01,
                    median: float = 64.0, sigma: float = 1.2, lo: int = 1, hi: int = 65536, base: int = 0):
    """Batched workload: log-normal string lengths (median 64 B, sigma 1.2, clipped to 1 B..64 KiB)."""
    lens = lengths(n_strings, "lognormal", median, sigma, lo, hi, seed)
    return batch_from_lengths(lens, variant, seed, err_frac, base)


def pareto_batch(n_strings: int, seed: int, xm: float = 1024.0, alpha: float = 1.1,
                 hi: int = 64 << 20, err_frac: float = 0.005, variants=("ascii", "latin", "cjk", "emoji")):
    """Heavy-tail workload: Pareto lengths (alpha 1.1, x_m 1 KiB, clipped at 64 MiB), per-string variant."""
    lens = lengths(n_strings, "pareto", xm, alpha, int(xm), hi, seed)
    rng = np.random.default_rng(_mix(seed, 9))
    var = [variants[i] for i in rng.integers(0, len(variants), size=n_strings)]
    return batch_from_lengths(lens, var, seed, err_frac)
