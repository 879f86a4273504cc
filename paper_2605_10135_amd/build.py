"""Compile the HIP sources under csrc/ into libsg.so for gfx950.

Each translation unit is compiled to an object in parallel, then linked into a
shared library next to this file.  Always rebuilds (the caller decides when).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsg.so")
BUILD_DIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(HERE, "..", "include")]


# Slices of the distance-kernel shape table (shapes.hip is compiled once per
# slice): precision x selection width, single-shard and batched.
PRECS = ("SG_PREC_FP32", "SG_PREC_F16", "SG_PREC_BF16", "SG_PREC_FP8", "SG_PREC_I8")
SLICES = [(p, k, 0) for p in PRECS for k in (32, 64, 128, 256)] + \
         [(p, k, 1) for p in PRECS for k in (64, 128, 256)]


def sources():
    """(source, object name, extra flags) of every translation unit."""
    units = [(os.path.join(CSRC, f), f + ".o", [])
             for f in sorted(os.listdir(CSRC)) if f.endswith(".hip") and f != "shapes.hip"]
    for p, k, b in SLICES:
        units.append((os.path.join(CSRC, "shapes.hip"), "shapes_%s_%s%d.o" % (p[8:].lower(), "b" if b else "r", k),
                      ["-DSG_SHAPE_PREC=" + p, "-DSG_SHAPE_KSEL=%d" % k, "-DSG_SHAPE_BATCHED=%d" % b]))
    # longest first (the shape slices), so that the pool finishes together
    return sorted(units, key=lambda u: os.path.basename(u[0]) not in ("shapes.hip",))


def _compile(unit) -> str:
    src, name, extra = unit
    obj = os.path.join(BUILD_DIR, name)
    cmd = [HIPCC] + FLAGS + extra + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sources()
    workers = min(len(srcs), max(1, os.cpu_count() or 1), 16)
    with cf.ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
