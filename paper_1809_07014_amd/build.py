"""Build the HIP library ``libkmerhip.so`` in-tree for gfx950.

Each ``csrc/*.hip`` file is compiled by hipcc into an object (in parallel) and
the objects are linked into one shared library next to this file.  Packed
FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
SO = os.path.join(HERE, "libkmerhip.so")
BUILD_DIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I" + INCLUDE, "-I" + CSRC]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip"))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    return obj


def build_library(verbose: bool = False) -> str:
    """Compile every HIP source and link ``libkmerhip.so``; returns its path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr)
    os.replace(tmp, SO)
    if verbose:
        print("built", SO)
    return SO


MICRO_SRC = os.path.join(HERE, "microbench", "roofline.hip")
MICRO_BIN = os.path.join(HERE, "microbench", "roofline")


def build_microbench() -> str:
    """Compile the roofline microbenchmark executable (not part of the
    library; used to measure the copy / random-access / atomic ceilings)."""
    tmp = MICRO_BIN + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-O3", "--offload-arch=" + ARCH, "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-o", tmp, MICRO_SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (MICRO_SRC, r.stderr))
    os.replace(tmp, MICRO_BIN)
    return MICRO_BIN


if __name__ == "__main__":
    build_library(verbose=True)
    build_microbench()
