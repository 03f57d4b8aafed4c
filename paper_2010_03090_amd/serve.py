"""Serving loop bindings: a continuous-batching validation server and its load replay.

The server and the replay driver are native (``csrc/serve.hip``); this module
marshals arguments.  Requests live in pinned host memory (torch tensors made
with ``pin_memory=True``): the GPU reads their payloads and offsets and writes
their results directly.
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._native import ServerConfig, Utf8vError, check, load

MODE_SERVER, MODE_PER_REQUEST = 0, 1


def default_config(**kw) -> ServerConfig:
    c = ServerConfig()
    check(load().utf8v_server_default_config(ctypes.byref(c)), "utf8v_server_default_config")
    for k, v in kw.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, int(v))
    return c


class Request:
    """One request in pinned host memory: strings data[offsets[k]:offsets[k+1]], result arrays."""

    def __init__(self, data: np.ndarray, offsets: np.ndarray):
        import torch
        n = offsets.size - 1
        self.n = n
        self.data = torch.empty(max(int(data.size), 1), dtype=torch.uint8, pin_memory=True)
        self.data[: data.size].copy_(torch.from_numpy(np.ascontiguousarray(data)))
        self.offsets = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int64)).pin_memory()
        self.flags = torch.full((max(n, 1),), 7, dtype=torch.uint8, pin_memory=True)
        self.first_err = torch.full((max(n, 1),), -7, dtype=torch.int64, pin_memory=True)

    @property
    def bytes(self) -> int:
        return int(self.offsets[-1] - self.offsets[0])

    def results(self):
        return self.flags[: self.n].numpy().copy(), self.first_err[: self.n].numpy().copy()

    def reset(self):
        self.flags.fill_(7)
        self.first_err.fill_(-7)


class Server:
    """Continuous-batching server on the current device (use as a context manager)."""

    def __init__(self, cfg: ServerConfig | None = None):
        self._lib = load()
        self.cfg = cfg or default_config()
        h = ctypes.c_void_p()
        check(self._lib.utf8v_server_create(ctypes.byref(self.cfg), ctypes.byref(h)), "utf8v_server_create")
        self._h = h

    def submit(self, req: Request) -> int:
        t = ctypes.c_uint64()
        check(self._lib.utf8v_server_submit(self._h, req.data.data_ptr(), req.offsets.data_ptr(), req.n,
                                            req.flags.data_ptr(), req.first_err.data_ptr(), ctypes.byref(t)),
              "utf8v_server_submit")
        return int(t.value)

    def poll(self, ticket: int) -> bool:
        return check(self._lib.utf8v_server_poll(self._h, ticket, None), "utf8v_server_poll") == 1

    def wait(self, ticket: int) -> int:
        done = ctypes.c_int64()
        check(self._lib.utf8v_server_wait(self._h, ticket, ctypes.byref(done)), "utf8v_server_wait")
        return int(done.value)

    def stats(self) -> dict:
        out = (ctypes.c_int64 * 4)()
        check(self._lib.utf8v_server_stats(self._h, out), "utf8v_server_stats")
        return {"requests_done": out[0], "batches": out[1], "largest_batch": out[2], "ring_bytes": out[3]}

    def close(self) -> None:
        if self._h:
            h, self._h = self._h, None
            check(self._lib.utf8v_server_destroy(h), "utf8v_server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def poisson_arrivals(rate_per_s: float, n: int, seed: int) -> np.ndarray:
    """Arrival times (ns from the start) of an open-loop Poisson process."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1e9 / rate_per_s, n)
    return np.cumsum(gaps).astype(np.int64)


def replay(pool: list[Request], arrivals_ns: np.ndarray, picks: np.ndarray, mode: int,
           cfg: ServerConfig | None = None) -> tuple[np.ndarray, int]:
    """Play the schedule (native, open loop); returns (latency ns per request, span ns)."""
    lib = load()
    cfg = cfg or default_config()
    k = len(pool)
    P = ctypes.c_void_p * k
    data = P(*[r.data.data_ptr() for r in pool])
    offs = P(*[r.offsets.data_ptr() for r in pool])
    ns = (ctypes.c_int64 * k)(*[r.n for r in pool])
    flags = P(*[r.flags.data_ptr() for r in pool])
    errs = P(*[r.first_err.data_ptr() for r in pool])
    arr = np.ascontiguousarray(arrivals_ns, dtype=np.int64)
    pk = np.ascontiguousarray(picks, dtype=np.int32)
    lat = np.zeros(arr.size, dtype=np.int64)
    span = ctypes.c_int64(0)
    rc = lib.utf8v_serve_replay(ctypes.byref(cfg), mode, data, offs, ns, flags, errs, k, arr.ctypes.data,
                                pk.ctypes.data, arr.size, lat.ctypes.data, ctypes.byref(span))
    if rc:
        raise Utf8vError(rc, "utf8v_serve_replay")
    return lat, int(span.value)
