#!/usr/bin/env python3
"""Benchmark of the MI355X lookup UTF-8 validator (one JSON line on stdout).

Headline workload (the single-buffer configuration of the metric): 1 GiB
buffers of synthetic text, five seeded variants -- pure ASCII, Latin-like
(85% 1-byte / 15% 2-byte), CJK-like (10% 1-byte / 90% 3-byte), emoji-heavy
(40% 1-byte / 60% 4-byte) and uniform random bytes -- plus, for each valid
variant, a copy with one error in its last 4 bytes.  One step validates all
nine buffers once (9 GiB); buffers are resident in HBM before timing starts.

Also reported: the measured read ceiling of the same buffers (a plain OR
reduction, the GPU analogue of the paper's memcpy column), the batched
workload (1,000,000 log-normal strings) against one launch per string, and the
CPU oracle on a bounded sample (a baseline, not a target).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "validated GB/s & % HBM peak (1 GiB buffer); batched strings/s; p99 latency"
HBM_PEAK_GBPS = 8000.0        # MI355X published HBM3E bandwidth
GIB = 1 << 30
VARIANTS = [("ascii", 1), ("latin", 2), ("cjk", 3), ("emoji", 4), ("random", 5)]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--warmup-seconds", type=float, default=0.5,
                    help="keep warming up until this much time passed (engine clocks ramp up under load)")
    ap.add_argument("--no-single", action="store_true", help="skip the single-buffer part (batch profiling)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also copy one buffer (profiling: scales the HBM traffic counters)")
    ap.add_argument("--per-string", type=int, default=10_000,
                    help="strings in the one-launch-per-string baseline (0 skips it)")
    ap.add_argument("--size", type=int, default=GIB, help="bytes per single buffer")
    ap.add_argument("--batch-strings", type=int, default=1_000_000)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="bounded oracle sample time")
    ap.add_argument("--variants", default="ascii,latin,cjk,emoji,random",
                    help="comma list of single-buffer variants (profiling runs restrict this)")
    ap.add_argument("--no-tail-copies", action="store_true", help="skip the copies with a tail error")
    ap.add_argument("--config", default="", help="launch overrides, e.g. unroll=4,waves_per_cu=24,ascii=1")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-loop part")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph / small-batch launch comparison")
    ap.add_argument("--no-heavy", action="store_true", help="skip the heavy-tail batches")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch configuration")
    ap.add_argument("--no-copy", action="store_true", help="skip the fused copy + validate part")
    ap.add_argument("--no-latency", action="store_true", help="skip the 1 MiB latency part")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper-shaped random inputs")
    ap.add_argument("--serve-loads", default="10000,50000,200000", help="offered loads, requests/s")
    ap.add_argument("--serve-requests", type=int, default=100_000, help="measured requests per load")
    ap.add_argument("--serve-baseline-requests", type=int, default=20_000,
                    help="measured requests per load for one synchronous launch per request")
    ap.add_argument("--serve-pool", type=int, default=256, help="distinct pre-generated requests")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (a single buffer would shard "
              "into contiguous byte ranges with a 3-byte halo and one minimum reduction; batches by "
              "string ranges with no exchange)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU (MI355X)", file=sys.stderr)
        sys.exit(1)
    import paper_2010_03090_amd as u8
    from paper_2010_03090_amd import synth
    lib = u8.load()
    if args.config:
        u8.set_config(**{k: int(v) for k, v in (kv.split("=") for kv in args.config.split(","))})
        args.no_autotune = True
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream or None

    if args.no_single:
        result = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "data": "synthetic"}
        host = {}
    else:
        result, host = bench_single(u8, lib, synth, torch, dev, stream, sh, args)

    # ---- batched: 1M log-normal strings vs one launch per string ------------------------------
    if not args.no_batch:
        result["batched"] = bench_batch(u8, lib, synth, torch, dev, stream, sh, args)

    # ---- latency of one 1 MiB buffer (the mixed-text correctness workload) ----------------------
    if not args.no_latency:
        result["latency_1mib"] = bench_latency(u8, lib, synth, torch, dev, stream, sh)

    # ---- fused copy + validate (device to device, pinned host to device) ----------------------
    if not args.no_copy:
        result["copy_validate"] = bench_copy(u8, synth, torch, dev, stream, args)

    # ---- heavy-tail batches: 20,000 Pareto strings, ~125 MiB and ~4 GiB ------------------------
    if not args.no_batch and not args.no_heavy:
        result["batched_heavy_tail"] = bench_heavy(u8, lib, synth, torch, dev, stream, sh, args)

    # ---- the paper's randomized inputs: 65,536 strings of 16 KiB per byte-length mix ------------
    if not args.no_batch and not args.no_paper:
        result["paper_shaped"] = bench_paper_shaped(u8, lib, synth, torch, dev, stream, sh, args)

    # ---- serving: continuous batching under Poisson load vs one launch per request -----------
    if not args.no_serve:
        result["serving"] = bench_serving(synth, args)

    # ---- CPU oracle on a bounded sample (1 core, as the paper's single thread) -----------------
    if not args.no_cpu and "random" in host and len(host) > 1:
        result["cpu_baseline"] = cpu_baseline(host, args.size, args.cpu_seconds)
        result["host_simd_lookup"] = host_simd_baseline(host, args.size)
    print(json.dumps(result), flush=True)


def recorded_traffic():
    """HBM bytes per 1 GiB launch from the committed rocprofv3 FETCH/WRITE summary, or None.

    The figure is used only while the kernel sources hash to the value recorded
    with it; any change to them makes it stale (None).
    """
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", "single_main_1gib.md")).read()
        rec = dict(l.split(": ", 1) for l in text.splitlines() if l.startswith(("traffic_bytes", "source_sha")))
        src = "".join(open(os.path.join(ROOT, "paper_2010_03090_amd", "csrc", f)).read()
                      for f in ("single.hip", "lookup.hpp", "common.hpp"))
        if hashlib.sha256(src.encode()).hexdigest() != rec["source_sha256"].strip():
            return None
        return int(rec["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def bench_single(u8, lib, synth, torch, dev, stream, sh, args):
    # ---- inputs (generated on the host, copied to HBM before timing) ---------------------
    n = args.size
    t0 = time.time()
    bufs, names, expected = [], [], []
    host = {}
    chosen = [v for v in VARIANTS if v[0] in args.variants.split(",")]
    for name, seed in chosen:
        h = synth.text(n, name, seed)
        host[name] = h
        bufs.append(torch.from_numpy(h).to(dev))
        names.append(name)
        expected.append(None)
    for name, seed in ([] if args.no_tail_copies else [v for v in chosen if v[0] != "random"]):
        t = bufs[names.index(name)].clone()
        tail, s, cls = synth.tail_error_copy(host[name][-64:], seed)
        t[-64:].copy_(torch.from_numpy(tail))
        bufs.append(t)
        names.append(name + "+tail_error")
        expected.append(s + n - 64)
    torch.cuda.synchronize()
    log(f"inputs ready in {time.time() - t0:.1f}s: {len(bufs)} x {n} bytes")

    # correctness gate (the oracle checks are in tests/; here the generator's known answers,
    # and for the random bytes the answer before timing, which every timed call must repeat)
    for i, (name, t, e) in enumerate(zip(names, bufs, expected)):
        got = u8.first_error(t)
        if e is not None and got != e:
            raise SystemExit(f"wrong result on {name}: {got} != {e}")
        if e is None and name != "random" and got != -1:
            raise SystemExit(f"wrong result on {name}: {got} != -1")
        expected[i] = got

    tuned = None if args.no_autotune else autotune_single(u8, lib, bufs[:len(chosen)])

    out = torch.empty(len(bufs), dtype=torch.int64, device=dev)
    ptrs = [t.data_ptr() for t in bufs]
    outp = [out.data_ptr() + 8 * i for i in range(len(bufs))]
    validate_async = lib.utf8v_validate_async

    def step(events=None):
        for i, p in enumerate(ptrs):
            if events is not None:
                events[i][0].record(stream)
            rc = validate_async(p, n, outp[i], sh)
            if events is not None:
                events[i][1].record(stream)
            if rc:
                raise u8.Utf8vError(rc, "utf8v_validate_async")

    # ---- read ceiling on the same buffers -------------------------------------------------
    ro = torch.zeros(1, dtype=torch.int32, device=dev)
    base_bufs = bufs[:len(chosen)]
    for _ in range(2):
        for t in base_bufs:
            u8.read_ceiling(t, ro)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 5
    ev[0].record(stream)
    for _ in range(reps):
        for t in base_bufs:
            u8.read_ceiling(t, ro)
    ev[1].record(stream)
    torch.cuda.synchronize()
    read_gbps = reps * len(base_bufs) * n / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e9

    # ---- headline: K timed steps ----------------------------------------------------------
    t_w = time.perf_counter()
    done = 0
    while done < args.warmup or time.perf_counter() - t_w < args.warmup_seconds:
        step()
        torch.cuda.synchronize()
        done += 1
    # whole-job throughput: K steps back to back, nothing else on the stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-launch durations for the roofline: the same K steps with events around every launch
    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
            for _ in bufs] for _ in range(args.steps)]
    torch.cuda.synchronize()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    if args.copy_probe:
        dst = torch.empty_like(bufs[0])
        for _ in range(3):
            u8.copy(bufs[0], dst)
        torch.cuda.synchronize()
        del dst
    res = out.cpu().numpy()
    for name, e, r in zip(names, expected, res):
        if e is not None and r != e:
            raise SystemExit(f"wrong timed result on {name}")
    per = np.array([[evs[k][i][0].elapsed_time(evs[k][i][1]) for i in range(len(bufs))]
                    for k in range(args.steps)]) * 1e-3          # seconds
    total_bytes = args.steps * len(bufs) * n
    value = total_bytes / wall / 1e9
    avg_launch = float(per.mean())
    achieved = n / avg_launch / 1e9
    per_variant = {names[i]: round(n / float(np.median(per[:, i])) / 1e9, 1) for i in range(len(bufs))}
    log("per-variant GB/s:", per_variant, "read ceiling GB/s:", round(read_gbps, 1))

    result = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "single-buffer validate, 1 GiB x (" + ", ".join(v for v, _ in chosen) + ")"
                               + ("" if args.no_tail_copies else " + copies with an error in the last 4 bytes")
                               + " per step",
                   "bytes_per_buffer": n, "buffers_per_step": len(bufs),
                   "launch": u8.get_config()},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": recorded_traffic() if n == GIB else None,
                     "traffic_unit": "bytes per 1 GiB launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE, "
                                     "profiles/single_main_1gib.md)",
                     "kernel": "single_main per 1 GiB launch (one launch per buffer), HIP events"},
        "pct_hbm_peak": round(100 * value / HBM_PEAK_GBPS, 1),
        "read_ceiling_GBps": round(read_gbps, 1),
        "pct_of_read_ceiling": round(100 * value / read_gbps, 1),
        "per_variant_GBps": per_variant,
        "per_variant_launch_us": {names[i]: {"min": round(float(per[:, i].min()) * 1e6, 1),
                                             "median": round(float(np.median(per[:, i])) * 1e6, 1),
                                             "mean": round(float(per[:, i].mean()) * 1e6, 1)}
                                  for i in range(len(bufs))},
        "GiBps": round(total_bytes / wall / GIB, 1),
        "autotune": tuned,
    }

    return result, host


def _top(cands, ms, k=4):
    order = np.argsort(ms)[:k]
    return [{"config": cands[i], "ms": round(float(ms[i]), 4)} for i in order]


def autotune_single(u8, lib, bufs, rounds=7):
    """The native autotuner on the benchmark's own 1 GiB buffers (one of each variant)."""
    import ctypes
    P = ctypes.c_void_p * len(bufs)
    S = ctypes.c_size_t * len(bufs)
    best = u8.Config()
    times = (ctypes.c_float * 64)()
    t0 = time.time()
    k = lib.utf8v_autotune_single(P(*[b.data_ptr() for b in bufs]), S(*[b.numel() for b in bufs]), len(bufs),
                                  rounds, ctypes.byref(best), times, 64)
    if k < 0:
        raise u8.Utf8vError(k, "utf8v_autotune_single")
    cands = [f"unroll={u},waves_per_cu={w},ascii={a}" for u in (2, 4, 8) for w in (8, 12, 16, 20, 24, 32, 40)
             for a in (0, 1)]
    ms = np.array([times[i] for i in range(k)])
    log(f"autotuned single-buffer launch in {time.time() - t0:.1f}s: {best.as_dict()}")
    return {"chosen": {f: best.as_dict()[f] for f in ("unroll", "waves_per_cu", "ascii")}, "rounds": rounds,
            "fastest_ms_for_all_buffers": _top(cands, ms)}


def _batch_launch(u8):
    c = u8.get_config()
    return {k: c[k] for k in ("batch_waves_per_cu", "batch_ascii", "batch_unroll")}


def autotune_batch(u8, lib, td, to, n, flags, ferr, rounds=7):
    import ctypes
    best = u8.Config()
    times = (ctypes.c_float * 64)()
    k = lib.utf8v_autotune_batch(td.data_ptr(), to.data_ptr(), n, flags.data_ptr(), ferr.data_ptr(), rounds,
                                 ctypes.byref(best), times, 64)
    if k < 0:
        raise u8.Utf8vError(k, "utf8v_autotune_batch")
    cands = [f"batch_waves_per_cu={w},batch_ascii={a},batch_unroll={u}"
             for w in (4, 8, 12, 16, 20, 24, 32, 48, 64) for a in (0, 1) for u in (4, 8)]
    ms = np.array([times[i] for i in range(k)])
    log(f"autotuned batch launch: {best.as_dict()}")
    return {"chosen": {"batch_waves_per_cu": best.batch_waves_per_cu, "batch_ascii": best.batch_ascii,
                       "batch_unroll": best.batch_unroll},
            "rounds": rounds, "fastest_ms_x3": _top(cands, ms)}


def bench_batch(u8, lib, synth, torch, dev, stream, sh, args):
    t0 = time.time()
    data, offsets, expected = synth.lognormal_batch(args.batch_strings, 2)
    td = torch.from_numpy(data).to(dev)
    to = torch.from_numpy(offsets).to(dev)
    flags = torch.empty(args.batch_strings, dtype=torch.uint8, device=dev)
    ferr = torch.empty(args.batch_strings, dtype=torch.int64, device=dev)
    log(f"batch inputs ready in {time.time() - t0:.1f}s: {data.size} bytes")
    fn = lib.utf8v_validate_batch_async
    nstr = args.batch_strings
    tuned = None
    if not args.no_autotune:  # tuned on a batch of the same shape from another seed
        t_data, t_off, _ = synth.lognormal_batch(args.batch_strings, 12)
        t_td, t_to = torch.from_numpy(t_data).to(dev), torch.from_numpy(t_off).to(dev)
        tuned = autotune_batch(u8, lib, t_td, t_to, nstr, flags, ferr)
        tuned["tuning_seed"] = 12
        del t_data, t_off, t_td, t_to

    def run():
        rc = fn(td.data_ptr(), to.data_ptr(), nstr, flags.data_ptr(), ferr.data_ptr(), sh)
        if rc:
            raise u8.Utf8vError(rc, "utf8v_validate_batch_async")

    t_w = time.perf_counter()
    while time.perf_counter() - t_w < args.warmup_seconds:
        run()
        torch.cuda.synchronize()
    got = ferr.cpu().numpy()
    if not np.array_equal(got[expected >= 0], expected[expected >= 0]) or (got[expected < 0] != -1).any():
        raise SystemExit("wrong batch result")
    reps = max(5, args.steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    blocks = []  # median of five timed blocks of back-to-back launches
    for _ in range(5):
        e0.record(stream)
        for _ in range(reps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        blocks.append(e0.elapsed_time(e1) * 1e-3 / reps)
    warm = float(np.median(blocks))
    # cold: evict the MALL with a 1 GiB read between timed runs
    scratch = torch.empty(GIB, dtype=torch.uint8, device=dev)
    ro = torch.zeros(1, dtype=torch.int32, device=dev)
    cold = []
    for _ in range(5):
        u8.read_ceiling(scratch, ro)
        e0.record(stream)
        run()
        e1.record(stream)
        torch.cuda.synchronize()
        cold.append(e0.elapsed_time(e1) * 1e-3)
    cold_t = float(np.median(cold))
    del scratch
    # baseline: one launch per string (validate_async per string) on a subsample
    sub = args.per_string
    per_string = None
    if sub > 0:
        outs = torch.empty(sub, dtype=torch.int64, device=dev)
        va = lib.utf8v_validate_async
        base = td.data_ptr()
        offs = offsets[:sub + 1]
        op = outs.data_ptr()
        for k in range(min(200, sub)):
            va(base + int(offs[k]), int(offs[k + 1] - offs[k]), op + 8 * k, sh)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(sub):
            va(base + int(offs[k]), int(offs[k + 1] - offs[k]), op + 8 * k, sh)
        torch.cuda.synchronize()
        per_string = sub / (time.perf_counter() - t0)
        if not np.array_equal(outs.cpu().numpy(), expected[:sub]):
            raise SystemExit("wrong per-string result")
    graph = None if args.no_graph else bench_graph(u8, lib, torch, td, to, flags, ferr, nstr, offsets, expected,
                                                   stream, sh, reps, warm)
    payload = int(offsets[-1] - offsets[0])
    algo = payload + 17 * nstr   # payload + offsets (8 B) + flag (1 B) + first_err (8 B) per string
    return {"workload": "1,000,000 strings, log-normal lengths (median 64 B, sigma 1.2, 1 B..64 KiB), "
                        "mixed code points, 1% injected errors",
            "strings_per_s_warm": round(nstr / warm), "strings_per_s_cold": round(nstr / cold_t),
            "ms_warm": round(warm * 1e3, 3), "ms_cold": round(cold_t * 1e3, 3),
            "ms_warm_blocks": [round(b * 1e3, 4) for b in blocks],
            "payload_GBps_warm": round(payload / warm / 1e9, 1),
            "algorithmic_GBps_warm": round(algo / warm / 1e9, 1),
            "per_string_launch_strings_per_s": round(per_string) if per_string else None,
            "speedup_vs_per_string_launch": round(nstr / warm / per_string, 1) if per_string else None,
            "graph": graph, "autotune": tuned, "launch": _batch_launch(u8)}


def bench_graph(u8, lib, torch, td, to, flags, ferr, nstr, offsets, expected, stream, sh, reps, warm):
    """The same batch through the captured-graph entry point, and small batches direct vs graph."""
    direct, graphed = lib.utf8v_validate_batch_async, lib.utf8v_validate_batch_graph

    def call(fn, n):
        rc = fn(td.data_ptr(), to.data_ptr(), n, flags.data_ptr(), ferr.data_ptr(), sh)
        if rc:
            raise u8.Utf8vError(rc, "batch")

    ferr.fill_(-7)
    call(graphed, nstr)
    torch.cuda.synchronize()
    got = ferr.cpu().numpy()
    if not np.array_equal(got[expected >= 0], expected[expected >= 0]) or (got[expected < 0] != -1).any():
        raise SystemExit("wrong graph batch result")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        call(graphed, nstr)
    e1.record(stream)
    torch.cuda.synchronize()
    g_warm = e0.elapsed_time(e1) * 1e-3 / reps
    out = {"ms_warm_1m": round(g_warm * 1e3, 3), "ms_warm_1m_direct": round(warm * 1e3, 3)}
    for n in (64, 4096):
        row = {}
        for name, fn in (("direct", direct), ("graph", graphed)):
            for _ in range(50):
                call(fn, n)
            torch.cuda.synchronize()
            k = 2000
            t0 = time.perf_counter()
            for _ in range(k):
                call(fn, n)
            torch.cuda.synchronize()
            row[f"{name}_us_per_call_pipelined"] = round((time.perf_counter() - t0) / k * 1e6, 2)
            lat = []
            for _ in range(300):
                t0 = time.perf_counter()
                call(fn, n)
                torch.cuda.synchronize()
                lat.append(time.perf_counter() - t0)
            row[f"{name}_us_latency_p50"] = round(float(np.median(lat)) * 1e6, 1)
            if not np.array_equal(ferr[:n].cpu().numpy()[expected[:n] >= 0], expected[:n][expected[:n] >= 0]):
                raise SystemExit(f"wrong {name} small-batch result")
        out[f"n{n}"] = row
    return out


def bench_latency(u8, lib, synth, torch, dev, stream, sh):
    """1 MiB of mixed text (and 64 corrupted copies): host-measured latency of a synchronous
    validate (launch, kernel, result copy, wait), and pipelined launches per second."""
    import ctypes
    clean, copies = synth.single_buffer_with_errors(1 << 20, "mixed", 0, 64)
    bufs = [torch.from_numpy(clean).to(dev)] + [torch.from_numpy(c).to(dev) for c, _, _ in copies]
    expect = [-1] + [int(s) for _, s, _ in copies]
    out = ctypes.c_int64(0)
    lat = []
    for rep in range(30):
        for t, e in zip(bufs, expect):
            t0 = time.perf_counter()
            lib.utf8v_validate_ex(t.data_ptr(), t.numel(), ctypes.byref(out), sh)
            lat.append(time.perf_counter() - t0)
            if out.value != e:
                raise SystemExit("wrong 1 MiB result")
    lat = np.array(lat[len(bufs):]) * 1e6
    res = torch.empty(len(bufs), dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 20
    for _ in range(reps):
        for i, t in enumerate(bufs):
            lib.utf8v_validate_async(t.data_ptr(), t.numel(), res.data_ptr() + 8 * i, sh)
    torch.cuda.synchronize()
    per = (time.perf_counter() - t0) / (reps * len(bufs))
    if res.cpu().numpy().tolist() != expect:
        raise SystemExit("wrong pipelined 1 MiB result")
    return {"workload": "1 MiB mixed text + 64 copies with one injected error each",
            "sync_latency_us_p50": round(float(np.percentile(lat, 50)), 1),
            "sync_latency_us_p99": round(float(np.percentile(lat, 99)), 1),
            "pipelined_us_per_buffer": round(per * 1e6, 2),
            "pipelined_GBps_cache_resident": round((1 << 20) / per / 1e9, 1)}


def bench_copy(u8, synth, torch, dev, stream, args):
    """1 GiB of CJK-like text: copy alone, validate alone, copy then validate, and the fused pass;
    from device memory and from pinned host memory."""
    n = GIB
    h = synth.text(n, "cjk", 3)
    src_d = torch.from_numpy(h).to(dev)
    src_h = torch.from_numpy(h).pin_memory()
    dst = torch.empty(n, dtype=torch.uint8, device=dev)
    out = torch.empty(2, dtype=torch.int64, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    reps = max(5, args.steps // 2)
    t_w = time.perf_counter()
    while time.perf_counter() - t_w < args.warmup_seconds:
        u8.copy_validate(src_d, dst, out[0:1])
        torch.cuda.synchronize()
    row = {"bytes": n}
    t_copy = timed(lambda: u8.copy(src_d, dst), reps)
    t_rt_copy = timed(lambda: dst.copy_(src_d), reps)   # the runtime's device-to-device copy
    t_val = timed(lambda: u8.validate_async(src_d, out[1:2]), reps)
    t_both = timed(lambda: (u8.copy(src_d, dst), u8.validate_async(src_d, out[1:2])), reps)
    t_fused = timed(lambda: u8.copy_validate(src_d, dst, out[0:1]), reps)
    if int(out[0]) != -1 or not torch.equal(dst[-4096:], src_d[-4096:]):
        raise SystemExit("wrong copy_validate result")
    row["device_to_device_GBps"] = {"copy": round(n / t_copy / 1e9, 1), "runtime_copy": round(n / t_rt_copy / 1e9, 1),
                                    "validate": round(n / t_val / 1e9, 1),
                                    "copy_then_validate": round(n / t_both / 1e9, 1),
                                    "fused": round(n / t_fused / 1e9, 1)}
    t_h2d = timed(lambda: dst.copy_(src_h, non_blocking=True), 3)
    t_h2d_val = timed(lambda: (dst.copy_(src_h, non_blocking=True), u8.validate_async(dst, out[1:2])), 3)
    t_h_fused = timed(lambda: u8.copy_validate(src_h, dst, out[0:1]), 3)
    if int(out[0]) != -1:
        raise SystemExit("wrong host copy_validate result")
    row["pinned_host_to_device_GBps"] = {"copy": round(n / t_h2d / 1e9, 1),
                                         "copy_then_validate": round(n / t_h2d_val / 1e9, 1),
                                         "fused": round(n / t_h_fused / 1e9, 1)}
    log(f"copy+validate GB/s: {row}")
    del src_d, src_h, dst
    torch.cuda.empty_cache()
    return row


def bench_heavy(u8, lib, synth, torch, dev, stream, sh, args):
    """20,000 strings, Pareto lengths (alpha 1.1, clipped at 64 MiB), per-string valid variant, 0.5% errors.

    x_m = 1 KiB gives ~125 MiB in total; x_m = 34 KiB gives ~4 GiB.  Each batch's launch
    shape is autotuned on a batch of the same shape from another seed (unless
    --no-autotune); timed through the direct
    launch and the captured-graph entry point.  The launch configuration is restored
    afterwards.
    """
    rows = []
    saved = u8.get_config()
    for name, xm in (("xm_1KiB", 1024.0), ("xm_34KiB", 34 * 1024.0)):
        t0 = time.time()
        data, offsets, expected = synth.pareto_batch(20_000, 3, xm=xm)
        td = torch.from_numpy(data).to(dev)
        to = torch.from_numpy(offsets).to(dev)
        del data
        n = offsets.size - 1
        flags = torch.empty(n, dtype=torch.uint8, device=dev)
        ferr = torch.empty(n, dtype=torch.int64, device=dev)
        log(f"heavy-tail {name}: {int(offsets[-1]) / 2**20:.0f} MiB ready in {time.time() - t0:.1f}s")
        row = {"workload": name, "payload_bytes": int(offsets[-1] - offsets[0]),
               "largest_string": int(np.diff(offsets).max())}
        u8.set_config(**saved)
        if not args.no_autotune:  # tuned on a batch of the same shape from another seed
            t_data, t_off, _ = synth.pareto_batch(20_000, 13, xm=xm)
            t_td, t_to = torch.from_numpy(t_data).to(dev), torch.from_numpy(t_off).to(dev)
            t_n = t_off.size - 1
            t_flags = torch.empty(t_n, dtype=torch.uint8, device=dev)
            t_ferr = torch.empty(t_n, dtype=torch.int64, device=dev)
            row["autotune"] = autotune_batch(u8, lib, t_td, t_to, t_n, t_flags, t_ferr)
            row["autotune"]["tuning_seed"] = 13
            del t_data, t_off, t_td, t_to, t_flags, t_ferr
            torch.cuda.empty_cache()
        row["launch"] = _batch_launch(u8)
        for mode, fn in (("direct", lib.utf8v_validate_batch_async), ("graph", lib.utf8v_validate_batch_graph)):
            def run():
                rc = fn(td.data_ptr(), to.data_ptr(), n, flags.data_ptr(), ferr.data_ptr(), sh)
                if rc:
                    raise u8.Utf8vError(rc, mode)
            ferr.fill_(-7)
            t_w = time.perf_counter()
            while time.perf_counter() - t_w < args.warmup_seconds:
                run()
                torch.cuda.synchronize()
            if not np.array_equal(ferr.cpu().numpy(), expected):
                raise SystemExit(f"wrong heavy-tail result ({name}, {mode})")
            reps = max(5, args.steps // 2)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                run()
            e1.record(stream)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) * 1e-3 / reps
            row[mode] = {"ms": round(t * 1e3, 3), "payload_GBps": round(row["payload_bytes"] / t / 1e9, 1),
                         "strings_per_s": round(n / t)}
        rows.append(row)
        del td, to, flags, ferr
        torch.cuda.empty_cache()
    u8.set_config(**saved)
    return rows


def bench_paper_shaped(u8, lib, synth, torch, dev, stream, sh, args):
    """The paper's randomized inputs (section 7.3): strings of 16 KiB whose code points have a
    byte length uniform over {1}, {1,2}, {1,2,3} or {1,2,3,4}; 65,536 of them (1 GiB) per mix,
    validated as one batch (each string its own stream, as each input is in the paper).  The
    paper's single-core figures for these inputs are context only (other hardware, in-cache).
    """
    rows = []
    n, length = 65536, 16384
    flags = torch.empty(n, dtype=torch.uint8, device=dev)
    ferr = torch.empty(n, dtype=torch.int64, device=dev)
    saved = u8.get_config()
    tuned = None
    if not args.no_autotune:  # tuned on a batch of the same shape (mix {1,2}) from another seed
        t_data, t_off, _ = synth.batch_from_lengths(np.full(n, length, np.int64), "unif2", 60)
        t_td, t_to = torch.from_numpy(t_data).to(dev), torch.from_numpy(t_off).to(dev)
        tuned = autotune_batch(u8, lib, t_td, t_to, n, flags, ferr)
        tuned["tuning_seed"] = 60
        del t_data, t_off, t_td, t_to
        torch.cuda.empty_cache()
    launch = _batch_launch(u8)
    for i, variant in enumerate(("unif1", "unif2", "unif3", "unif4")):
        data, offsets, _ = synth.batch_from_lengths(np.full(n, length, np.int64), variant, 40 + i)
        td = torch.from_numpy(data).to(dev)
        to = torch.from_numpy(offsets).to(dev)
        del data

        def run():
            rc = lib.utf8v_validate_batch_async(td.data_ptr(), to.data_ptr(), n, flags.data_ptr(),
                                                ferr.data_ptr(), sh)
            if rc:
                raise u8.Utf8vError(rc, "utf8v_validate_batch_async")
        ferr.fill_(-7)
        t_w = time.perf_counter()
        while time.perf_counter() - t_w < args.warmup_seconds:
            run()
            torch.cuda.synchronize()
        if not bool((ferr == -1).all()):
            raise SystemExit(f"wrong paper-shaped result ({variant})")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        blocks = []
        for _ in range(3):
            e0.record(stream)
            for _ in range(5):
                run()
            e1.record(stream)
            torch.cuda.synchronize()
            blocks.append(e0.elapsed_time(e1) * 1e-3 / 5)
        t = float(np.median(blocks))
        rows.append({"variant": variant, "ms": round(t * 1e3, 3), "GBps": round(n * length / t / 1e9, 1),
                     "GiBps": round(n * length / t / 2**30, 1)})
        log(f"paper-shaped {variant}: {rows[-1]['GBps']} GB/s")
        del td, to
        torch.cuda.empty_cache()
    u8.set_config(**saved)
    return {"workload": "65,536 strings x 16 KiB per byte-length mix (one batch, all valid)",
            "autotune": tuned, "launch": launch, "results": rows}


def bench_serving(synth, args):
    """Open-loop Poisson arrivals; each request 1..4096 strings shaped like the 1M-string batch.

    Payloads are pre-generated in pinned host memory (a pool of distinct requests,
    replayed); host-to-device copies are inside the measured latency.  Latency =
    results on the host - scheduled arrival.  1 s of warm-up arrivals precede the
    measured ones at each load.
    """
    from paper_2010_03090_amd import serve
    t0 = time.time()
    rng = np.random.default_rng(2024)
    pool, expect, bytes_, strings_ = [], [], [], []
    for i in range(args.serve_pool):
        m = int(rng.integers(1, 4097))
        lens = synth.lengths(m, "lognormal", 64, 1.2, 1, 65536, 7000 + i)
        data, offsets, known = synth.batch_from_lengths(lens, "mixed", 9000 + i, err_frac=0.01)
        pool.append(serve.Request(data, offsets))
        # the generator's own answers (valid text, one injected error at a known offset)
        expect.append(((known < 0).astype(np.uint8), known))
        bytes_.append(int(offsets[-1]))
        strings_.append(m)
    bytes_, strings_ = np.array(bytes_), np.array(strings_)
    log(f"serving pool ready in {time.time() - t0:.1f}s: {len(pool)} requests, mean {bytes_.mean() / 1e3:.0f} KB, "
        f"{strings_.mean():.0f} strings")
    loads = []
    for li, rate in enumerate(int(x) for x in args.serve_loads.split(",")):
        row = {"offered_req_per_s": rate, "offered_GBps": round(rate * bytes_.mean() / 1e9, 2)}
        for mode, name, nmeas in ((serve.MODE_SERVER, "continuous_batching", args.serve_requests),
                                  (serve.MODE_PER_REQUEST, "per_request_launch", args.serve_baseline_requests)):
            nwarm = int(min(rate * 1.0, nmeas))
            n = nwarm + nmeas
            arrivals = serve.poisson_arrivals(rate, n, 100 + li)
            picks = np.random.default_rng(200 + li).integers(0, len(pool), n)
            for r in pool:
                r.reset()
            t1 = time.time()
            lat, span = serve.replay(pool, arrivals, picks, mode)
            for k in set(picks.tolist()):
                f, e = pool[k].results()
                if not (np.array_equal(e, expect[k][1]) and np.array_equal(f, expect[k][0])):
                    raise SystemExit(f"wrong serving result ({name}, load {rate}, request {k})")
            m_lat = lat[nwarm:] / 1e3
            mp = picks[nwarm:]
            # measured window: first measured arrival to last completion
            win = (arrivals[-1] - arrivals[nwarm] + lat[-1]) / 1e9
            done_bytes = float(bytes_[mp].sum())
            row[name] = {"p50_us": round(float(np.percentile(m_lat, 50)), 1),
                         "p99_us": round(float(np.percentile(m_lat, 99)), 1),
                         "mean_us": round(float(m_lat.mean()), 1),
                         "achieved_req_per_s": round(nmeas / win),
                         "GBps": round(done_bytes / win / 1e9, 2),
                         "strings_per_s": round(float(strings_[mp].sum()) / win),
                         "requests": nmeas, "warmup_requests": nwarm}
            log(f"serving {name} at {rate}/s: p50 {row[name]['p50_us']} us, p99 {row[name]['p99_us']} us, "
                f"{row[name]['GBps']} GB/s ({time.time() - t1:.1f}s)")
        loads.append(row)
    return {"workload": "Poisson arrivals; each request 1..4096 strings (uniform), log-normal lengths "
                        "(median 64 B, sigma 1.2), mixed code points, 1% injected errors; payloads in pinned "
                        "host memory, copies included",
            "admission_budget_bytes": int(serve.default_config().budget_bytes),
            "pool_requests": len(pool), "mean_request_bytes": round(float(bytes_.mean())),
            "loads": loads}


def cpu_baseline(host, n, seconds):
    """The oracle, single-threaded (the paper's protocol), on bounded prefixes of the valid variants.

    The random-bytes variant is reported apart: the branchy walk stops at its
    first error a few bytes in, while the GPU scans the whole buffer.
    """
    import oracle
    per_variant = {}
    total_b, total_t = 0, 0.0
    valid = [k for k in host if k != "random"]
    budget = seconds / len(valid)
    for name in valid:
        h = host[name]
        size = 1 << 24
        done_b, done_t = 0, 0.0
        while done_t < budget and done_b < n:
            seg = h[done_b: done_b + size]
            t0 = time.perf_counter()
            oracle.first_error(seg)
            done_t += time.perf_counter() - t0
            done_b += seg.size
        per_variant[name] = round(done_b / done_t / 1e9, 3)
        total_b += done_b
        total_t += done_t
    t0 = time.perf_counter()
    r = oracle.first_error(host["random"])
    per_variant["random(stops at offset %d)" % r] = round(n / (time.perf_counter() - t0) / 1e9, 1)
    try:
        cpu = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
    except Exception:
        cpu = platform.processor()
    mib = total_b / len(valid) / (1 << 20)
    return {"value": round(total_b / total_t / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"branchy oracle on 1 thread over the first ~{mib:.0f} MiB of each valid variant buffer "
                      f"(ascii, latin, cjk, emoji; 16 MiB segments, ~{budget:.1f} s each)",
            "per_variant_GBps": per_variant, "host_cpu": cpu, "host_threads": os.cpu_count()}


def host_simd_baseline(host, n):
    """The section 6 lookup algorithm with AVX2 on the host (the paper's own method on a CPU),
    1 thread and all threads, on the valid variant buffers.  A reference point only."""
    from paper_2010_03090_amd import baselines
    if not baselines.supported():
        return None
    threads = min(os.cpu_count() or 1, 64)
    row = {"unit": "GB/s", "threads_all": threads}
    for label, nt in (("one_thread", 1), ("all_threads", threads)):
        per = {}
        for name in (k for k in host if k != "random"):
            h = host[name][: n if nt > 1 else min(n, 256 << 20)]
            baselines.is_valid(h[: 1 << 20], nt)
            t0 = time.perf_counter()
            ok = baselines.is_valid(h, nt)
            per[name] = round(h.size / (time.perf_counter() - t0) / 1e9, 2)
            if not ok:
                raise SystemExit(f"host lookup baseline rejected valid {name}")
        row[label] = per
    return row


if __name__ == "__main__":
    main()
