"""Builds the HIP library ``libfsa.so`` for gfx950, in-tree.

Usage: ``python -m paper_2504_19410_amd.build [--force]``.  Every source under
``csrc/`` is compiled by hipcc as HIP C++ (object files in ``_build/``) and
linked into ``paper_2504_19410_amd/libfsa.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libfsa.so")
ARCH = os.environ.get("FSA_OFFLOAD_ARCH", "gfx950")

SOURCES = [
    "fsa_api.cpp",
    "fsa_batch.cpp",
    "fsa_server.cpp",
    "fsa_tensor.hip",
    "fsa_spectral.hip",
    "fsa_dd.hip",
    "fsa_tune.cpp",
    "fsa_launch_f32_v0.hip",
    "fsa_launch_f32_v1.hip",
    "fsa_launch_f32_v2.hip",
    "fsa_launch_f32_v3.hip",
    "fsa_launch_f32_v4.hip",
    "fsa_launch_f64_v0.hip",
    "fsa_launch_f64_v1.hip",
    "fsa_launch_f64_v2.hip",
    "fsa_launch_f64_v3.hip",
    "fsa_launch_f64_v4.hip",
]

CXXFLAGS = [
    "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _headers():
    return [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))] + [
        os.path.join(os.path.dirname(PKG), "include", "fsa.h")]


def _compile(src: str, force: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if not force and os.path.exists(obj):
        newest = max(os.path.getmtime(p) for p in [path] + _headers())
        if os.path.getmtime(obj) >= newest:
            return obj
    cmd = ["hipcc", *CXXFLAGS, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(force: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), SOURCES))
    if force or not os.path.exists(LIB) or any(
            os.path.getmtime(o) > os.path.getmtime(LIB) for o in objs):
        tmp = LIB + ".tmp"
        cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
               "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stderr}")
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
