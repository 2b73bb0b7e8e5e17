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
           "batch.cpp", "static_sweep.hip", "kernels_rows.hip"]
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


def _deps_mtime(path: str, seen=None) -> float:
    """Newest modification time of a source and the local headers it includes."""
    import re

    seen = set() if seen is None else seen
    if path in seen or not os.path.exists(path):
        return 0.0
    seen.add(path)
    t = os.path.getmtime(path)
    with open(path) as fh:
        for inc in re.findall(r'^\s*#\s*include\s+"([^"]+)"', fh.read(), flags=re.M):
            t = max(t, _deps_mtime(os.path.normpath(os.path.join(os.path.dirname(path), inc)), seen))
    return t


def build(verbose: bool = True, incremental: bool = False) -> str:
    """Compile every source and link the shared library.  By default every
    object is rebuilt; with incremental=True only objects older than their
    source or a local header it includes are."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        path = os.path.join(CSRC, src)
        if incremental and os.path.exists(obj) and os.path.getmtime(obj) > _deps_mtime(path):
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
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs,
           # roctx ranges around the sweep calls (a no-op without a profiler)
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv, incremental="--incremental" in sys.argv)
