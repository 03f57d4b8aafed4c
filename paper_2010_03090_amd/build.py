"""Build the gfx950 validator library (``libutf8v.so``) and the helper C libraries in-tree.

    python -m paper_2010_03090_amd.build          # compile everything
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libutf8v.so")
BUILD = os.path.join(PKG, "_build")
SOURCES = ["single.hip", "batch.hip", "misc.hip", "serve.hip", "tune.hip", "api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         # no packed-FP32 instructions anywhere in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    subprocess.check_call([HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj],
                          stderr=subprocess.STDOUT if False else None)
    return obj


def build_hip() -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, OUT)
    return OUT


def build_all() -> None:
    sys.path.insert(0, ROOT)
    from paper_2010_03090_amd import synth
    synth.build(force=True)
    build_hip()


if __name__ == "__main__":
    build_all()
    print(OUT)
