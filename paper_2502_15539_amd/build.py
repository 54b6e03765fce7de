"""Compile the HIP library (gfx950) in-tree: paper_2502_15539_amd/libptrhash_hip.so."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libptrhash_hip.so")
OBJDIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("PTRHASH_ARCH", "gfx950")

HIP_SOURCES = ["api.hip", "kernels.hip", "roofline.hip", "keygen.hip", "server.hip", "build_device.hip",
               "place_device.hip", "noalloc.hip"]
CXX_SOURCES = ["builder.cpp"]

# Packed FP32 instructions are kept out of every HIP object on purpose.
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]
CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-I", INCLUDE, "-I", CSRC,
             "-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    """Compile every source (always, even if a library exists) and link."""
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = [(["hipcc", *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", os.path.join(OBJDIR, src + ".o")],
             os.path.join(OBJDIR, src + ".o")) for src in HIP_SOURCES]
    jobs += [(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", os.path.join(OBJDIR, src + ".o")],
              os.path.join(OBJDIR, src + ".o")) for src in CXX_SOURCES]
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "0")) or (os.cpu_count() or 1), 8))
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda j: _run(j[0]), jobs))
    objs = [o for _, o in jobs]
    tmp = LIB + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
