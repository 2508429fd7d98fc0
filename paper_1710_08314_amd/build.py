"""Build step of the gfx950 decoder library (libpolar_scl.so, in-tree).

hipcc cross-compiles for gfx950 without a GPU.  Device code is built without
packed-FP32 instructions and without floating-point contraction (the float32
decoder must round every f/g and penalty exactly as written), and with uniform
control-flow regions left unstructured (scalar branches).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libpolar_scl.so")
BUILD_DIR = os.path.join(PKG, "_build")

HIP_SOURCES = ["decode.hip", "sc.hip", "scx.hip", "rq.hip", "rq10.hip", "rq9.hip", "gen.hip",
               "noalloc.hip"]
# Per-file flags.  rq.hip keeps a path's whole state in registers, reached
# through a switch over tree levels; merging the cases' common stores would
# turn those registers into stack memory.
_RQ_FLAGS = ["-mllvm", "-simplifycfg-sink-common=false"]
EXTRA = {"rq.hip": _RQ_FLAGS, "rq10.hip": _RQ_FLAGS, "rq9.hip": _RQ_FLAGS}
CPP_SOURCES = ["plan.cpp", "capi.cpp", "server.cpp"]

ARCH = os.environ.get("POLAR_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-strict-aliasing", "-Wall",
          "-Wno-unused-function"]
# The decoder's op dispatch is uniform control flow (every lane of a wave runs
# the same node program); leaving uniform regions to scalar branches instead
# of the structurizer's flag variables saves scalar and vector instructions.
DEVICE = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-fno-gpu-flush-denormals-to-zero", "-munsafe-fp-atomics",
          "-mllvm", "-structurizecfg-skip-uniform-regions"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"compile failed: {cmd[-1]}")
    return r


def build(verbose: bool = False) -> str:
    """Compile every HIP/C++ source and link libpolar_scl.so (always rebuilds)."""
    hipcc = _hipcc()
    os.makedirs(BUILD_DIR, exist_ok=True)
    inc = ["-I", CSRC, "-I", os.path.join(os.path.dirname(PKG), "include")]
    objs = []
    jobs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        jobs.append([hipcc, *COMMON, *DEVICE, *EXTRA.get(src, []), *inc, "-c",
                     os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in CPP_SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        jobs.append([hipcc, *COMMON, *inc, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    procs = [subprocess.Popen(j, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
             for j in jobs]
    failed = []
    for j, p in zip(jobs, procs):
        out, err = p.communicate()
        if verbose and (out or err):
            sys.stderr.write(out + err)
        if p.returncode != 0:
            failed.append((j, out + err))
    if failed:
        for j, msg in failed:
            sys.stderr.write(" ".join(j) + "\n" + msg)
        raise RuntimeError("compile failed")
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
