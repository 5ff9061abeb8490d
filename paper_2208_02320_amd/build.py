"""Build the gfx950 HIP library ``libhh.so`` in place (next to this file).

Every ``csrc/*.hip`` translation unit is compiled by ``hipcc`` for gfx950 in
parallel, then linked into one shared library that exports the C ABI of
``include/hh.h``.  Also builds ``calib/copy``, the plain copy kernel used to
calibrate profiler byte counters, and ``examples/hh_client``, a plain C client
of the ABI.  Run as ``python -m paper_2208_02320_amd.build``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.environ.get("HH_BUILD_DIR", os.path.join(ROOT, "_build"))
LIB = os.environ.get("HH_LIB_OUT", os.path.join(HERE, "libhh.so"))
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for all device code.  Multiply-adds
# are fused only within one source expression (-ffp-contract=on), never
# across statements, so every instantiation of a kernel template (tile
# variants of one axis pass) rounds the same arithmetic the same way and the
# variants give identical bits.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=on"]
COMMON = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wno-unused-command-line-argument",
          "-I", os.path.join(ROOT, "include")] + os.environ.get("HH_EXTRA_FLAGS", "").split()


def _compile(src, obj):
    cmd = [HIPCC] + COMMON + DEVICE_FLAGS + ["-c", src, "-o", obj]
    t = time.time()
    p = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (p.stderr or "").splitlines() if "packed-fp32-ops" not in l
                    and "warning: unknown target feature" not in l)
    if p.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), err))
    return os.path.basename(src), time.time() - t


def build(jobs=None, verbose=True):
    """Compile every HIP source and link libhh.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    objs = [os.path.join(BUILD, os.path.basename(s)[:-4] + ".o") for s in srcs]
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for name, dt in ex.map(lambda so: _compile(*so), zip(srcs, objs)):
            if verbose:
                print("  hipcc %-22s %6.1fs" % (name, dt), flush=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lz"]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), p.stderr))
    os.replace(tmp, LIB)
    calib = os.path.join(HERE, "calib", "copy.cpp")
    exe = os.path.join(HERE, "calib", "copy")
    cmd = [HIPCC, "-x", "hip"] + COMMON + DEVICE_FLAGS + [calib, "-o", exe + ".tmp"]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("calibration kernel build failed: %s\n%s" % (" ".join(cmd), p.stderr))
    os.replace(exe + ".tmp", exe)
    if LIB == os.path.join(HERE, "libhh.so"):
        build_client()
    if verbose:
        print("built %s in %.1fs" % (LIB, time.time() - t0), flush=True)
    return LIB


def build_client():
    """The plain C client of the ABI (examples/hh_client.c), linked against
    libhh.so with gcc; it finds the library next to itself at run time."""
    src = os.path.join(HERE, "examples", "hh_client.c")
    exe = os.path.join(HERE, "examples", "hh_client")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), src,
           "-L", HERE, "-lhh", "-Wl,-rpath,$ORIGIN/..", "-o", exe + ".tmp"]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("C client build failed: %s\n%s" % (" ".join(cmd), p.stderr))
    os.replace(exe + ".tmp", exe)
    return exe


if __name__ == "__main__":
    build(jobs=int(sys.argv[1]) if len(sys.argv) > 1 else None)
