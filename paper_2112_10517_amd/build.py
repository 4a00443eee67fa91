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


# the compiler's per-kernel resource report (registers, spills, scratch,
# LDS, occupancy) of every device function, kept beside the library
RESOURCES = os.path.join(OUTDIR, "resource_usage.txt")


def _compile(src: str, objdir: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(objdir, src + ".o")
    cmd = [HIPCC] + COMMON + DEVICE + ["-Rpass-analysis=kernel-resource-usage", "-x", "hip", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-6000:]))
    with open(obj + ".resources", "w") as f:
        f.write(r.stderr)
    return obj


def resource_report(objs) -> dict:
    """{kernel symbol: {field: value}} from the compiler remarks of the objects."""
    import re
    out, cur = {}, None
    for obj in objs:
        with open(obj + ".resources") as f:
            for line in f:
                m = re.search(r"remark: Function Name: (\S+)", line)
                if m:
                    cur = out.setdefault(m.group(1), {})
                    continue
                m = re.search(r"remark:\s+([A-Za-z][A-Za-z /\[\]]*?): (\S+) \[-Rpass-analysis", line)
                if m and cur is not None:
                    cur[m.group(1).strip()] = m.group(2)
    return out


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
    rep = resource_report(objs)
    with open(RESOURCES + ".tmp", "w") as f:
        for name in sorted(rep):
            f.write(name + " " + " ".join("%s=%s" % (k.replace(" ", "_"), v) for k, v in sorted(rep[name].items()))
                    + "\n")
    os.replace(RESOURCES + ".tmp", RESOURCES)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
