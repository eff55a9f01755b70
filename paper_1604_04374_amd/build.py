"""Compile the HIP library ``libpc.so`` for gfx950 in-tree.

Usage: ``python -m paper_1604_04374_amd.build`` (or ``build()`` from Python).
Every call recompiles; translation units are built in parallel.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libpc.so")
BUILD_DIR = os.path.join(os.path.dirname(PKG), "_build")

SOURCES = ["kern_1d.hip", "kern_2d.hip", "kern_sec.hip", "kern_construct.hip", "kern_wavelet.hip", "pc_api.cpp",
           "tune.cpp"]
ARCH = "gfx950"
# Packed FP32 instructions are switched off for the device code (the
# compiler otherwise forms them from float / float2 arithmetic).
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function"]
# extra compiler flags for tuning experiments (e.g. -DPC_LDS_PAD=32)
COMMON += os.environ.get("PC_EXTRA_FLAGS", "").split()


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _filter(out: str) -> str:
    # the host pass does not know the device-only target feature; drop that note
    keep = [l for l in out.splitlines() if "packed-fp32-ops" not in l]
    return "\n".join(keep)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()
    t0 = time.time()
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = [cc, *COMMON, *DEVICE_FLAGS, "-I", os.path.join(os.path.dirname(PKG), "include"),
               "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = []
    for src, cmd, p in procs:
        out, _ = p.communicate()
        out = _filter(out)
        if p.returncode != 0:
            failed.append((src, " ".join(cmd), out))
        elif verbose and out.strip():
            print(out)
    if failed:
        msg = "\n\n".join(f"[{s}] {c}\n{o}" for s, c, o in failed)
        raise RuntimeError(f"HIP compilation failed:\n{msg}")
    tmp = OUT + ".tmp"
    cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{_filter(r.stdout)}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} in {time.time() - t0:.1f}s")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
