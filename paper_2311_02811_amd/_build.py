"""Build libcontour.so (HIP for gfx950) in-tree with hipcc.

Each source compiles to an object in parallel, then one link makes the
shared library next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(PKG, "libcontour.so")

SOURCES = [
    "contour_runtime.cpp",
    "contour_single.hip",
    "contour_batch.hip",
    "contour_reorder.hip",
    "contour_serve.cpp",
    "contour_noalloc.hip",
    "contour_merge.hip",
]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return path


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed: %s\n%s%s" % (" ".join(cmd), res.stdout, res.stderr))
    return res.stdout + res.stderr


def build(verbose: bool = False) -> str:
    """Compile every source into paper_2311_02811_amd/libcontour.so (always rebuilds)."""
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="contour_build_") as tmp:
        objs, cmds = [], []
        for src in SOURCES:
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            objs.append(obj)
            cmds.append([cc, *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", "-o", obj,
                         os.path.join(CSRC, src)])
        workers = min(len(cmds), max(1, os.cpu_count() or 1))
        with ThreadPoolExecutor(workers) as ex:
            logs = list(ex.map(_run, cmds))
        out = LIB_PATH + ".tmp%d" % os.getpid()
        logs.append(_run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out, *objs]))
    if verbose:
        print("".join(logs))
    os.replace(out, LIB_PATH)
    return LIB_PATH
