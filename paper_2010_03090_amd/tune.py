"""Autotuner front end: sample inputs, the native timing search, and a per-device cache.

The search itself is native (``utf8v_autotune_single`` / ``utf8v_autotune_batch``):
it times every launch configuration in interleaved rounds on the GPU and keeps
the fastest.  This module draws the sample inputs (the workload shapes of the
benchmark, scaled down), and caches the chosen configuration in a JSON file
keyed by device, compute-unit count and library build, so later processes can
apply it without searching again.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os

import numpy as np

from . import synth
from ._native import LIB_PATH, Config, Utf8vError, check, load

CACHE_ENV = "UTF8V_TUNE_CACHE"


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "utf8v", "tune.json")


def device_key() -> dict:
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    with open(LIB_PATH, "rb") as f:
        lib_sha = hashlib.sha256(f.read()).hexdigest()[:16]
    return {"device": props.name, "arch": getattr(props, "gcnArchName", ""), "cus": int(load().utf8v_num_cus()),
            "library": lib_sha}


def read_cache(path: str | None = None) -> list:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, list) else []
    except (OSError, ValueError):
        return []


def lookup(key: dict, entries: list) -> dict | None:
    for e in entries:
        if e.get("key") == key and isinstance(e.get("config"), dict):
            return e["config"]
    return None


def store(key: dict, config: dict, timings: dict, path: str | None = None) -> None:
    path = path or cache_path()
    entries = [e for e in read_cache(path) if e.get("key") != key]
    entries.append({"key": key, "config": config, "timings": timings})
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1)
    os.replace(tmp, path)


def apply_cached(path: str | None = None) -> dict | None:
    """Set the cached configuration for this device and build, if there is one; returns it."""
    from . import set_config
    cfg = lookup(device_key(), read_cache(path))
    if cfg:
        set_config(**cfg)
    return cfg


def autotune(sample_mib: int = 256, batch_strings: int = 200_000, rounds: int = 7, seed: int = 0,
             cache: bool = True, path: str | None = None) -> dict:
    """Search both kernels' launch configurations on sample inputs; returns the chosen configuration."""
    import torch
    lib = load()
    n = sample_mib << 20
    bufs = [torch.from_numpy(synth.text(n, v, seed + i)).cuda() for i, v in enumerate(("mixed", "ascii", "cjk"))]
    P = ctypes.c_void_p * len(bufs)
    S = ctypes.c_size_t * len(bufs)
    best = Config()
    times = (ctypes.c_float * 64)()
    k = lib.utf8v_autotune_single(P(*[b.data_ptr() for b in bufs]), S(*[b.numel() for b in bufs]), len(bufs),
                                  rounds, ctypes.byref(best), times, 64)
    if k < 0:
        raise Utf8vError(k, "utf8v_autotune_single")
    single_ms = [round(float(times[i]), 4) for i in range(k)]
    del bufs
    data, offsets, _ = synth.lognormal_batch(batch_strings, seed + 7)
    td, to = torch.from_numpy(data).cuda(), torch.from_numpy(offsets).cuda()
    flags = torch.empty(batch_strings, dtype=torch.uint8, device="cuda")
    ferr = torch.empty(batch_strings, dtype=torch.int64, device="cuda")
    k2 = lib.utf8v_autotune_batch(td.data_ptr(), to.data_ptr(), batch_strings, flags.data_ptr(), ferr.data_ptr(),
                                  rounds, ctypes.byref(best), times, 64)
    if k2 < 0:
        raise Utf8vError(k2, "utf8v_autotune_batch")
    batch_ms = [round(float(times[i]), 4) for i in range(k2)]
    torch.cuda.synchronize()
    config = best.as_dict()
    if cache:
        store(device_key(), config, {"single_ms": single_ms, "batch_ms": batch_ms}, path)
    return config
