"""MI355X-native lookup UTF-8 validation (Keiser & Lemire, section 6) -- Python API.

Thin wrappers over the C-ABI of ``libutf8v.so``: PyTorch provides device
memory and streams, the library's HIP kernels do all the work.

    import torch, paper_2010_03090_amd as u8
    buf = torch.frombuffer(bytearray("héllo".encode()), dtype=torch.uint8).cuda()
    u8.validate(buf)                 # True
    u8.first_error(buf)              # -1
    flags, first_err = u8.validate_batch(data, offsets)   # CSR strings
"""
from __future__ import annotations

import ctypes

from . import _native
from ._native import Config, Utf8vError, check, load

__all__ = ["validate", "first_error", "validate_async", "validate_batch", "validate_batch_async",
           "validate_batch_graph", "Stream", "error_class", "error_classes", "ERROR_CLASSES", "copy_validate",
           "classify", "check_offsets", "get_config", "set_config", "num_cus", "read_ceiling", "copy",
           "Config", "Utf8vError", "load"]


def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> int | None:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    h = s.cuda_stream
    return h or None


def _dev_u8(t, name="buf"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA uint8 tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _dev_tensor(t, dtype, n: int, device, name: str):
    """t must be a contiguous CUDA tensor of `dtype` with at least n elements on `device`."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA {dtype} tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < n:
        raise ValueError(f"{name} holds {t.numel()} elements, {n} are written")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the input on {device}")
    return t


def _batch_args(data, offsets, flags, first_err) -> int:
    """Check a CSR batch call's tensors (all on one device); returns n."""
    torch = _torch()
    _dev_u8(data, "data")
    if not isinstance(offsets, torch.Tensor) or offsets.dtype != torch.int64 or not offsets.is_cuda \
            or offsets.numel() < 1:
        raise TypeError("offsets must be a CUDA int64 tensor with n+1 entries")
    if not offsets.is_contiguous():
        raise ValueError("offsets must be contiguous")
    if offsets.device != data.device:
        raise ValueError(f"offsets is on {offsets.device}, data on {data.device}")
    n = offsets.numel() - 1
    _dev_tensor(flags, torch.uint8, n, data.device, "flags")
    _dev_tensor(first_err, torch.int64, n, data.device, "first_err")
    return n


def first_error(buf, stream=None) -> int:
    """First-error offset of a CUDA uint8 tensor (-1 if it is valid UTF-8). Synchronizes the stream."""
    _dev_u8(buf)
    out = ctypes.c_int64(0)
    check(load().utf8v_validate_ex(buf.data_ptr() if buf.numel() else None, buf.numel(), ctypes.byref(out),
                                   _stream_handle(stream)), "utf8v_validate_ex")
    return int(out.value)


def validate(buf, stream=None) -> bool:
    """True iff the CUDA uint8 tensor holds valid UTF-8."""
    return first_error(buf, stream) < 0


def validate_async(buf, out, stream=None) -> None:
    """Enqueue validation; out (CUDA int64 tensor, 1 element) receives the first-error offset."""
    torch = _torch()
    _dev_u8(buf)
    _dev_tensor(out, torch.int64, 1, buf.device, "out")
    check(load().utf8v_validate_async(buf.data_ptr() if buf.numel() else None, buf.numel(), out.data_ptr(),
                                      _stream_handle(stream)), "utf8v_validate_async")


def validate_batch_async(data, offsets, flags, first_err, stream=None) -> None:
    """Enqueue the validation of CSR strings; flags (uint8) and first_err (int64) get n entries."""
    n = _batch_args(data, offsets, flags, first_err)
    if n == 0:
        return
    check(load().utf8v_validate_batch_async(data.data_ptr() if data.numel() else offsets.data_ptr(),
                                            offsets.data_ptr(), n, flags.data_ptr(), first_err.data_ptr(),
                                            _stream_handle(stream)), "utf8v_validate_batch_async")


def validate_batch_graph(data, offsets, flags, first_err, stream=None) -> None:
    """As validate_batch_async, launched as one replay of the per-stream captured HIP graph."""
    n = _batch_args(data, offsets, flags, first_err)
    if n == 0:
        return
    check(load().utf8v_validate_batch_graph(data.data_ptr() if data.numel() else offsets.data_ptr(),
                                            offsets.data_ptr(), n, flags.data_ptr(), first_err.data_ptr(),
                                            _stream_handle(stream)), "utf8v_validate_batch_graph")


def validate_batch(data, offsets, stream=None):
    """Validate CSR strings data[offsets[k]:offsets[k+1]]; returns (flags uint8, first_err int64) on the device.

    first_err is relative to each string start, -1 for valid strings.  The
    result tensors are ready when the given (or current) stream reaches them.
    """
    torch = _torch()
    _dev_u8(data, "data")
    n = offsets.numel() - 1
    flags = torch.empty(max(n, 0), dtype=torch.uint8, device=offsets.device)
    ferr = torch.empty(max(n, 0), dtype=torch.int64, device=offsets.device)
    validate_batch_async(data, offsets, flags, ferr, stream)
    return flags, ferr


def copy_validate(src, dst, out, stream=None) -> None:
    """Enqueue copy src -> dst (uint8 tensors, src may be pinned host memory) with validation in one pass.

    out (CUDA int64, 1 element) receives src's first-error offset (-1 if valid).
    """
    torch = _torch()
    if not isinstance(src, torch.Tensor) or src.dtype != torch.uint8 or not src.is_contiguous():
        raise TypeError("src must be a contiguous uint8 tensor (CUDA or pinned host)")
    _dev_u8(dst, "dst")
    if dst.numel() < src.numel():
        raise ValueError("dst is smaller than src")
    _dev_tensor(out, torch.int64, 1, dst.device, "out")
    check(load().utf8v_copy_validate(dst.data_ptr() if dst.numel() else None,
                                     src.data_ptr() if src.numel() else None, src.numel(), out.data_ptr(),
                                     _stream_handle(stream)), "utf8v_copy_validate")


ERROR_CLASSES = {0: "valid", 1: "five_plus_byte", 2: "too_short", 3: "too_long", 4: "overlong",
                 5: "too_large", 6: "surrogate"}


def error_class(buf, stream=None) -> int:
    """Section 3 rule (1..6 = a..f) broken by buf's first ill-formed character, 0 if valid. Synchronizes."""
    torch = _torch()
    _dev_u8(buf)
    fe = torch.empty(1, dtype=torch.int64, device=buf.device)
    cls = torch.empty(1, dtype=torch.uint8, device=buf.device)
    validate_async(buf, fe, stream)
    check(load().utf8v_error_class(buf.data_ptr() if buf.numel() else None, buf.numel(), fe.data_ptr(),
                                   cls.data_ptr(), _stream_handle(stream)), "utf8v_error_class")
    return int(cls.item())


def error_classes(data, offsets, first_err, stream=None):
    """Per-string class (uint8 tensor on the device) from a batch's first-error offsets."""
    torch = _torch()
    n = offsets.numel() - 1
    out = torch.empty(max(n, 0), dtype=torch.uint8, device=offsets.device)
    _batch_args(data, offsets, out, first_err)
    if n > 0:
        check(load().utf8v_error_classes(data.data_ptr() if data.numel() else offsets.data_ptr(),
                                         offsets.data_ptr(), n, first_err.data_ptr(), out.data_ptr(),
                                         _stream_handle(stream)), "utf8v_error_classes")
    return out


class Stream:
    """Validate one byte sequence fed in chunks (CUDA uint8 tensors); any split gives the whole's result.

    Keep each chunk alive until the next finish() (or synchronize the stream).
    """

    def __init__(self, stream=None):
        self._stream = stream
        h = ctypes.c_void_p()
        check(load().utf8v_stream_create(ctypes.byref(h), _stream_handle(stream)), "utf8v_stream_create")
        self._h = h
        self._keep = []

    def update(self, chunk) -> None:
        _dev_u8(chunk, "chunk")
        if chunk.numel() == 0:
            return
        check(load().utf8v_stream_update(self._h, chunk.data_ptr(), chunk.numel(), _stream_handle(self._stream)),
              "utf8v_stream_update")
        self._keep.append(chunk)

    def finish(self) -> int:
        """First-error offset of everything fed so far (-1 if valid); waits for the stream."""
        out = ctypes.c_int64(0)
        check(load().utf8v_stream_finish(self._h, ctypes.byref(out), _stream_handle(self._stream)),
              "utf8v_stream_finish")
        self._keep.clear()
        return int(out.value)

    @property
    def position(self) -> int:
        return int(load().utf8v_stream_position(self._h))

    def reset(self) -> None:
        check(load().utf8v_stream_reset(self._h, _stream_handle(self._stream)), "utf8v_stream_reset")

    def close(self) -> None:
        if self._h:
            _torch().cuda.current_stream().synchronize() if self._stream is None else self._stream.synchronize()
            check(load().utf8v_stream_destroy(self._h), "utf8v_stream_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def check_offsets(offsets, stream=None) -> bool:
    """True iff offsets (CUDA int64, n+1 entries) is non-decreasing from a non-negative start."""
    torch = _torch()
    _dev_tensor(offsets, torch.int64, 1, None, "offsets")
    n = offsets.numel() - 1
    return bool(check(load().utf8v_check_offsets(offsets.data_ptr(), n, _stream_handle(stream)),
                      "utf8v_check_offsets"))


def classify(buf, stream=None):
    """Per-position (classification byte, error byte) tensors of length len+1 (diagnostic)."""
    torch = _torch()
    _dev_u8(buf)
    sc = torch.empty(buf.numel() + 1, dtype=torch.uint8, device=buf.device)
    err = torch.empty_like(sc)
    check(load().utf8v_classify(buf.data_ptr() if buf.numel() else None, buf.numel(), sc.data_ptr(),
                                err.data_ptr(), _stream_handle(stream)), "utf8v_classify")
    return sc, err


def read_ceiling(buf, out, stream=None) -> None:
    check(load().utf8v_read_ceiling(buf.data_ptr(), buf.numel(), out.data_ptr(), _stream_handle(stream)),
          "utf8v_read_ceiling")


def copy(src, dst, stream=None) -> None:
    check(load().utf8v_copy(src.data_ptr(), dst.data_ptr(), src.numel(), _stream_handle(stream)), "utf8v_copy")


def get_config() -> dict:
    c = Config()
    check(load().utf8v_get_config(ctypes.byref(c)), "utf8v_get_config")
    return c.as_dict()


def set_config(**kw) -> dict:
    """Update launch parameters (unroll, waves_per_cu, ascii, batch_waves_per_cu, batch_ascii,
    batch_unroll)."""
    c = Config()
    check(load().utf8v_get_config(ctypes.byref(c)), "utf8v_get_config")
    for k, v in kw.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, int(v))
    check(load().utf8v_set_config(ctypes.byref(c)), "utf8v_set_config")
    return c.as_dict()


def num_cus() -> int:
    return int(load().utf8v_num_cus())
