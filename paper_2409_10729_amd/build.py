"""Build libmfx.so (HIP, gfx950) in-tree.

    python -m paper_2409_10729_amd.build

Each source compiles to its own object (in parallel: the kernel families
are instantiated in separate k_*.hip units), then hipcc links the shared
library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "libmfx.so")
SOURCES = ["mfx.hip", "learned.hip", "k_fp64.hip", "k_fp32.hip", "k_nf3_fp64.hip", "k_nf3_fp32.hip",
           "k_learned.hip", "k_xy_double.hip", "k_xy_float.hip", "k_xy_nf3.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

ARCH = ["--offload-arch=gfx950"]
FLAGS = ARCH + [
    "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions: the kernels are written for scalar FP32 issue
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _jobs() -> int:
    n = os.cpu_count() or 4
    for var in ("MAX_JOBS", "CMAKE_BUILD_PARALLEL_LEVEL"):
        if os.environ.get(var, "").isdigit():
            n = min(n, int(os.environ[var]))
    return max(1, min(n, len(SOURCES), 16))


def _compile(src: str, verbose: bool) -> tuple[str, subprocess.CompletedProcess]:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", "-o", obj, os.path.join(CSRC, src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    return obj, subprocess.run(cmd, capture_output=True, text=True)


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        results = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    failed = [(obj, r) for obj, r in results if r.returncode != 0]
    for obj, r in failed:
        sys.stderr.write(f"--- {obj}\n" + r.stdout + r.stderr)
    if failed:
        raise RuntimeError("hipcc failed compiling " + ", ".join(os.path.basename(o) for o, _ in failed))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, *ARCH, "-shared", "-fPIC", "-o", tmp, *[obj for obj, _ in results]]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libmfx.so")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
