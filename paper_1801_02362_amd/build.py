"""Build the HIP library (libpcv.so) for gfx950 and the host test library.

Run ``python -m paper_1801_02362_amd.build`` (or call ``build()``).  Objects go
to ``_build/`` at the repository root; the shared libraries are written next
to this file so that the package loads them in-tree.
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
BUILD = os.path.join(ROOT, "_build")
ARCH = os.environ.get("PCV_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}"]
# Packed FP32 instructions are disabled on purpose for all device code.
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]

SOURCES = ["pcv_kernels.hip", "pcv_engine2.hip", "pcv_engine3.hip", "pcv_engine4.hip", "pcv_api.hip", "pcv_batch.hip", "pcv_mlp.hip", "pcv_bias.hip", "pcv_nl.hip", "pcv_props.hip", "pcv_f2.hip", "pcv_ceiling.hip"]
LIB = os.path.join(PKG, "libpcv.so")
HOSTTEST_LIB = os.path.join(PKG, "libpcv_hosttest.so")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (r.stderr or "").splitlines() if noise not in l and l.strip() != "(ignoring feature)")
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{err}")
    return err


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    _run([HIPCC, *COMMON, *DEVICE, "-c", os.path.join(CSRC, src), "-o", obj])
    return obj


def build(verbose: bool = False) -> None:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    _run([HIPCC, *DEVICE, "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    tmp = HOSTTEST_LIB + ".tmp"
    _run([HIPCC, *COMMON, "-shared", "-o", tmp, os.path.join(CSRC, "pcv_hosttest.cpp")])
    os.replace(tmp, HOSTTEST_LIB)
    if verbose:
        print("built", LIB, HOSTTEST_LIB)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
