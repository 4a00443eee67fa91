"""Build the HIP library ``lib/libesdg.so`` for gfx950 in-tree.

Every translation unit under ``csrc/`` is compiled by hipcc in parallel and
linked into one shared library exporting the C ABI of ``include/esdg.h``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUTDIR = os.path.join(HERE, "lib")
LIB = os.path.join(OUTDIR, "libesdg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("ESDG_OFFLOAD_ARCH", "gfx950")

SOURCES = ["capi.hip", "batch.hip", "host_ops.cpp", "server.cpp", "dispatch_misc.hip", "dispatch_vol2d.hip",
           "dispatch_vol3d.hip", "dispatch_vol2d_f32.hip", "dispatch_vol3d_f32.hip", "dispatch_vol3d_tuned.hip",
           "dispatch_vol3d_f32_tuned.hip", "dispatch_vol3d_nodes.hip", "dispatch_vol3d_f32_nodes.hip",
           "dispatch_gauss.hip", "dispatch_gauss_f32.hip", "dispatch_vol3d_pairs.hip",
           "dispatch_vol3d_f32_pairs.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I", os.path.join(ROOT, "include")]
# Packed FP32 instructions are kept out of every device code object.
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _compile(src: str, objdir: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(objdir, src + ".o")
    cmd = [HIPCC] + COMMON + DEVICE + ["-x", "hip", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-6000:]))
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source (always) and link lib/libesdg.so; returns its path."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    os.makedirs(OUTDIR, exist_ok=True)
    jobs = min(len(SOURCES), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, objdir), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr[-4000:]))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
