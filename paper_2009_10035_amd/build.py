"""Build libf2v.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

Every translation unit is compiled in parallel, then linked into a shared
library next to this file.  Run `python -m paper_2009_10035_amd.build`.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libf2v.so")
ARCH = os.environ.get("F2V_OFFLOAD_ARCH", "gfx950")

SOURCES = [
    "f2v_kernels.hip",
    "f2v_variants_f32_v4.hip",
    "f2v_variants_f32_v2.hip",
    "f2v_variants_f32_v1.hip",
    "f2v_variants_bf16_v4.hip",
    "f2v_variants_bf16_v2.hip",
    "f2v_staged_f32_v1.hip",
    "f2v_staged_f32_v2.hip",
    "f2v_staged_bf16_v2.hip",
    "f2v_variants.cpp",
    "f2v_api.cpp",
    "f2v_server.cpp",
]
HEADERS = ["f2v_device.h", "f2v_kernels.h", "f2v_update_impl.h", "../../include/f2v.h"]

# -packed-fp32-ops: keep the compiler from emitting packed FP32 instructions.
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-x", "hip",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument"]


def _hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return exe


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{msgs}")
    if msgs:
        sys.stderr.write(msgs + "\n")
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    """Compile all sources (always) and link libf2v.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1), 16)
    t0 = time.time()
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True, capture_output=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
