"""Build the HIP library libffp.so for gfx950 in-tree with hipcc.

Run as ``python -m paper_2001_04109_amd.build`` (or through
``__graft_entry__.build()``).  Objects go to ``paper_2001_04109_amd/_build``;
the shared library lands next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libffp.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed-FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, *DEVICE_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, *COMMON, "-x", "hip", *DEVICE_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(jobs: int = 8, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


BUILD_ASAN = os.path.join(HERE, "_build_asan")
LIB_ASAN = os.path.join(HERE, "libffp_asan.so")


def _compile_host_asan(src: str) -> str:
    obj = os.path.join(BUILD_ASAN, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, "-x", "hip", "--offload-host-only", "-g", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fno-omit-frame-pointer", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc (host AddressSanitizer) failed for {src}:\n{r.stderr}")
    return obj


def build_host_asan(jobs: int = 8, verbose: bool = False) -> str:
    """libffp_asan.so: the host-side sources (*.cpp: planning, scheduling,
    the request loop, the autotuner's table, the C ABI) instrumented with
    AddressSanitizer, linked with the device objects of build().  For host
    tests only (load it with the sanitizer runtime preloaded and
    FFP_LIBRARY pointing at it); device code is not instrumented."""
    if not all(os.path.exists(os.path.join(BUILD, os.path.splitext(f)[0] + ".o")) for f in sources()):
        build(jobs=jobs)
    os.makedirs(BUILD_ASAN, exist_ok=True)
    host = [f for f in sources() if f.endswith(".cpp")]
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(host)))) as ex:
        hobjs = list(ex.map(_compile_host_asan, host))
    dobjs = [os.path.join(BUILD, os.path.splitext(f)[0] + ".o") for f in sources() if f.endswith(".hip")]
    tmp = LIB_ASAN + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *dobjs, *hobjs, "-Xarch_host",
           "-fsanitize=address", "-Xarch_host", "-shared-libasan", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link (host AddressSanitizer) failed:\n{r.stderr}")
    os.replace(tmp, LIB_ASAN)
    if verbose:
        print(f"built {LIB_ASAN}")
    return LIB_ASAN


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "asan":
        build_host_asan(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
