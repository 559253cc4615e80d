"""Host-side AddressSanitizer / UndefinedBehaviorSanitizer / LeakSanitizer run
of the C ABI (CPU only).

api.hip is compiled again with the sanitizers on its host code only (each
-fsanitize flag behind -Xarch_host; the device code is built as usual), linked
with the library's other objects into the driver tests/abi_host_check.c, and
run without a GPU: argument validation, workspace and scratch sizing for every
A form (including automatic rank and generic Fourier frames), refusals of null
handles and streams, the static-scratch size check of the allocation-free entry
point, and the error strings.  Any sanitizer report fails the run.
"""
import os
import shutil
import subprocess

import pytest

from paper_2311_03824_amd import build as B

OBJS = ["k_column.o", "k_column_tuned.o", "k_column_cached.o", "k_small.o", "k_gen.o", "k_fourier.o", "k_rank.o"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def test_abi_host_code_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    objs = [os.path.join(B.BUILD, o) for o in OBJS]
    missing = [o for o in objs if not os.path.exists(o)]
    if missing:
        pytest.skip(f"library objects not built (run __graft_entry__.build()): {missing}")
    api_o = str(tmp_path / "api_san.o")
    flags = [f"--offload-arch={B.ARCH}", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fno-omit-frame-pointer", "-I", B.INCLUDE, "-I", B.CSRC]
    res = subprocess.run([hipcc, *flags, *SAN, "-c", os.path.join(B.CSRC, "api.hip"), "-o", api_o],
                         capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-3000:]
    exe = str(tmp_path / "abi_check")
    here = os.path.dirname(os.path.abspath(__file__))
    res = subprocess.run([hipcc, f"--offload-arch={B.ARCH}", "-fPIC", *SAN, "-x", "c", "-I", B.INCLUDE,
                          os.path.join(here, "abi_host_check.c"), "-x", "none", api_o, *objs, "-o", exe],
                         capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    out = run.stdout + run.stderr
    assert run.returncode == 0 and "ok" in run.stdout, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out and "LeakSanitizer" not in out, out[-4000:]
