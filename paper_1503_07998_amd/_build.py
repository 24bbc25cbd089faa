"""Build the native library ``libmvd.so`` in-tree with hipcc for gfx950.

Every HIP source is compiled with packed-FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``); the host-side C++ is
compiled by hipcc as well.  Objects go to ``_build/`` next to this file and are
compiled in parallel.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import time
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmvd.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

ARCH = os.environ.get("MVD_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", f"-I{INCLUDE}", f"-I{CSRC}",
          "-Wall", "-Wno-unused-result", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the ROCm toolchain is required to build libmvd.so")
    return exe


# units that take longest to compile start first (the build is as long as its
# slowest unit plus whatever waited for a free worker)
_FIRST = ("k_sep_41", "k_sep_31", "k_sep_63", "k_pq", "k_sep_21", "k_sep_15", "k_fused", "k_adjoint")


def sources():
    names = [n for n in os.listdir(CSRC) if n.endswith((".hip", ".cpp"))]

    def rank(name):
        for i, p in enumerate(_FIRST):
            if name.startswith(p):
                return (i, name)
        return (len(_FIRST), name)

    return [os.path.join(CSRC, n) for n in sorted(names, key=rank)]


def _compile(src: str) -> tuple[str, float]:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [_hipcc(), *COMMON, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [_hipcc(), *COMMON, "-x", "hip", "-c", src, "-o", obj]
    t0 = time.perf_counter()
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n{res.stderr[-6000:]}")
    return obj, time.perf_counter() - t0


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every source and link ``libmvd.so``; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        done = list(ex.map(_compile, srcs))
    objs = [o for o, _ in done]
    if verbose:
        slow = sorted(zip(srcs, (t for _, t in done)), key=lambda st: -st[1])[:6]
        print("slowest: " + ", ".join(f"{os.path.basename(n)} {t:.0f} s" for n, t in slow), flush=True)
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr[-6000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(objs)} objects", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
