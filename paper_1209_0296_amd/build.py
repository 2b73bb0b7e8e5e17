"""Build the HIP library ``libspinlat.so`` in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libspinlat.so")
SOURCES = ["kernels_simple.hip", "kernels_stream.hip", "kernels_row.hip", "kernels_batch.hip",
           "kernels_ne_sub.hip", "kernels_ne_sub_b8.hip", "kernels_ne_sub_b16.hip",
           "kernels_ne_sub_b32.hip", "kernels_ne_sub_b64.hip", "host_logic.cpp", "runtime.cpp",
           "batch.cpp", "static_sweep.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 instructions stay off in every device build
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the host threshold table is evaluated without contraction
    "-ffp-contract=off", "-fno-fast-math",
    "-Wall", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _headers_mtime() -> float:
    paths = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".h", ".hpp"))]
    paths.append(os.path.join(ROOT, "include", "spinlat.h"))
    return max(os.path.getmtime(p) for p in paths)


def build(verbose: bool = True, incremental: bool = False) -> str:
    """Compile every source and link the shared library.  By default every
    object is rebuilt; with incremental=True only objects older than their
    source or any header are."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    hdr = _headers_mtime() if incremental else 0.0
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        path = os.path.join(CSRC, src)
        if incremental and os.path.exists(obj) and os.path.getmtime(obj) > max(
                hdr, os.path.getmtime(path)):
            continue
        cmd = [HIPCC, *FLAGS, "-c", path, "-o", obj]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        cmds.append(cmd)
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
        for rc, cmd in zip(ex.map(lambda c: subprocess.call(c), cmds), cmds):
            if rc != 0:
                raise subprocess.CalledProcessError(rc, cmd)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv, incremental="--incremental" in sys.argv)
