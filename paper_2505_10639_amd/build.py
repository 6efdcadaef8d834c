"""Build libmomfbd.so (gfx950) in-tree with hipcc.

Usage: python -m paper_2505_10639_amd.build   (or __graft_entry__.build()).
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmomfbd.so")
EMU = os.path.join(HERE, "libmomfbd_hostemu.so")

ARCH = "gfx950"
SOURCES = ["momfbd_api.hip", "kernels64.hip", "kernels96.hip", "kernels128.hip", "object.hip", "gemm_mfma.hip", "gemm_group.hip",
           "lbfgs.hip", "postproc.hip", "cnn.hip", "spectra.hip", "rng.hip"]
# Packed FP32 instructions are kept out of every code object; clang forms
# them from ordinary float code otherwise.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument", "-Wno-pass-failed"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_library(verbose: bool = True) -> str:
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    procs = []
    for src in SOURCES:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmd = [hipcc(), *HIP_FLAGS, "-I", CSRC, "-I", INCLUDE, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print("+", " ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    _run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


def build_hostemu(verbose: bool = True) -> str:
    """Host-only harness that runs the wave operators lane by lane on the CPU
    (test infrastructure; never loaded by the library binding)."""
    src = os.path.join(CSRC, "hostemu.cpp")
    tmp = EMU + ".tmp"
    cmd = [hipcc(), "-O2", "-std=c++17", "-fPIC", "-shared", "-x", "hip", "--offload-arch=" + ARCH,
           "-I", CSRC, "-I", INCLUDE, src, "-o", tmp]
    _run(cmd)
    os.replace(tmp, EMU)
    return EMU


def build_all():
    build_library()
    build_hostemu()


if __name__ == "__main__":
    build_all()
    sys.exit(0)
