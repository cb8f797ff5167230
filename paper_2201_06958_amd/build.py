"""Compile the HIP library (gfx950) in-tree: paper_2201_06958_amd/libtdb.so.

Every source is compiled with hipcc for gfx950 only, with packed FP32 instructions
disabled, into object files under <repo>/_build, then linked into one shared library
that exports the C ABI declared in include/tdb.h.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtdb.so")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = ["small_ops.hip", "stream_ops.hip", "dbo_ops.hip", "hosvd_ops.hip", "eig_ops.hip", "fused_ops.hip", "fused_pass.hip", "mfma_pass.hip", "gate_ops.hip",
           "noalloc_ops.hip", "rpass.hip",
           "tdb_api.cpp"]
ARCH = "gfx950"
FLAGS = ["-O3", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-fPIC", "-std=c++17", "-Wno-unused-result"]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc()] + FLAGS + ["-c", path, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [_hipcc(), "-x", "hip"] + FLAGS + ["-c", path, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{res.stderr[-4000:]}")
    return obj


def build_library(jobs: int = 4) -> str:
    """Compile every source and link libtdb.so; returns its path."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    res = subprocess.run([_hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs,
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr[-4000:]}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library())
