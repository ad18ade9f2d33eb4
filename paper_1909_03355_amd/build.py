"""Build libfedfem.so (HIP, gfx950) in-tree with hipcc, and the small
copy_calibrate program that scales the memory-traffic counters."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfedfem.so")
CALIB = os.path.join(HERE, "copy_calibrate")
SOURCES = ["fed_api.cpp", "fed_kernels.hip", "fed_tiling.cpp", "fed_lds_order.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # packed FP32 instructions stay off: plain scalar FP32 everywhere
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


def _hipcc(args, out, verbose):
    cmd = [HIPCC] + args + ["-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{err}")
    if verbose and err.strip():
        print(err)
    os.replace(out + ".tmp", out)


def build(verbose=False):
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    _hipcc(FLAGS + srcs, LIB, verbose)
    exe_flags = [f for f in FLAGS if f not in ("-fPIC", "-shared")]
    _hipcc(exe_flags + [os.path.join(CSRC, "copy_calibrate.hip")], CALIB, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
