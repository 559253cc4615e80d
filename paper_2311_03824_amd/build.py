"""Build libaltgdmin.so for gfx950 with hipcc (in-tree, no JIT cache).

Each .hip source is compiled in its own process (in parallel), then linked
into ``paper_2311_03824_amd/libaltgdmin.so``.  Run as
``python -m paper_2311_03824_amd.build`` or through ``__graft_entry__.build()``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libaltgdmin.so")
ARCH = os.environ.get("ALTGDMIN_ARCH", "gfx950")
# (source, extra flags, object): k_column.hip is compiled three times, the second
# time for the autotuned kernel variants only and the third for the cached-load
# instantiations, so the parts build in parallel.
SOURCES = [
    ("k_column.hip", ["-DALTG_PART=1"], "k_column.o"),
    ("k_column.hip", ["-DALTG_PART=2"], "k_column_tuned.o"),
    ("k_column.hip", ["-DALTG_PART=3"], "k_column_cached.o"),
    ("k_small.hip", [], "k_small.o"),
    ("k_gen.hip", [], "k_gen.o"),
    ("k_fourier.hip", [], "k_fourier.o"),
    ("k_rank.hip", [], "k_rank.o"),
    ("api.hip", [], "api.o"),
]

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def _hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def _compile(spec) -> str:
    src, extra, obj_name = spec
    obj = os.path.join(BUILD, obj_name)
    cmd = [_hipcc(), *HIPCC_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
