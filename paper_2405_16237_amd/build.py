"""Build the gfx950 shared library libnbvh.so in-tree with hipcc.

Every translation unit is compiled for gfx950 only, without floating-point
contraction (the slab test and the sample positions are defined one rounding
per operation), with correctly rounded single-precision division, hardware
FP32 atomics, and without packed-FP32 instruction selection.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libnbvh.so")
BUILD_DIR = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["api.hip", "kernels_traverse.hip", "kernels_query.hip", "kernels_train.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-fhip-fp32-correctly-rounded-divide-sqrt", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-6000:]))
    return obj


PEAKS_SRC = os.path.join(HERE, "peaks", "peaks.hip")
PEAKS_OUT = os.path.join(HERE, "peaks", "libnbvh_peaks.so")


def build_peaks(verbose: bool = False) -> str:
    """The ceiling micro-benchmarks (a separate library: not part of the
    N-BVH path)."""
    tmp = PEAKS_OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-shared", "-o", tmp, PEAKS_SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for peaks.hip:\n%s" % r.stderr[-4000:])
    os.replace(tmp, PEAKS_OUT)
    if verbose:
        print("built", PEAKS_OUT)
    return PEAKS_OUT


def build(verbose: bool = False) -> str:
    """Compile all sources and link libnbvh.so (always rebuilds), and the
    ceiling micro-benchmarks."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-4000:])
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    build_peaks(verbose)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
