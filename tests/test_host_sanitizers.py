"""Host AddressSanitizer and UndefinedBehaviorSanitizer over the C++ layer.

The library's host code (argument checks, plan tables, workspace carve and
the solver, network and spectrum set-up; the files whose host code only
sets up launches are taken from the regular build) and the host emulation
harness of the wave operators are rebuilt with -fsanitize=address,undefined
on the host side only, and the CPU tests of the boundary and of the
operators run against those builds in a child process with the sanitizer
runtime preloaded.  Any report fails.
"""

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2505_10639_amd")
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build", "sanitize")
# rebuilt with the sanitizers: every file with host logic beyond a launch
SANITIZED = ["momfbd_api.hip", "object.hip", "lbfgs.hip", "postproc.hip", "cnn.hip",
             "spectra.hip", "rng.hip"]
# taken from the regular build: host code that only sets up launches
REGULAR = ["kernels64.o", "kernels96.o", "kernels128.o", "gemm_mfma.o", "gemm_group.o"]
# host side only: each sanitizer flag applies to the host compilation
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer"]
COMMON = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", CSRC, "-I", os.path.join(ROOT, "include")]


def _hipcc():
    for cand in ("/opt/rocm/bin/hipcc",):
        if os.path.exists(cand):
            return cand
    pytest.skip("hipcc not available")


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        pytest.skip("clang AddressSanitizer runtime not found")
    return hits[-1]


def _build():
    os.makedirs(OUT, exist_ok=True)
    cc = _hipcc()

    def one(src):
        obj = os.path.join(OUT, src.replace(".hip", ".o"))
        subprocess.run([cc, *COMMON, *SAN, "-c", os.path.join(CSRC, src), "-o", obj],
                       check=True, capture_output=True)
        return obj

    regular = [os.path.join(PKG, "_build", o) for o in REGULAR]
    if not all(os.path.exists(o) for o in regular):
        from paper_2505_10639_amd import build
        build.build_library(verbose=False)
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(one, SANITIZED)) + regular
    lib = os.path.join(OUT, "libmomfbd_sanitized.so")
    subprocess.run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", *SAN, "-shared-libsan",
                    *objs, "-o", lib], check=True, capture_output=True)
    emu = os.path.join(OUT, "libmomfbd_hostemu_sanitized.so")
    # the harness has no device code; unoptimised, it builds in seconds
    subprocess.run([cc, "-O0", "-std=c++17", "-fPIC", "--offload-host-only", "-I", CSRC,
                    "-I", os.path.join(ROOT, "include"), *SAN, "-shared", "-shared-libsan",
                    "-x", "hip", os.path.join(CSRC, "hostemu.cpp"), "-o", emu],
                   check=True, capture_output=True)
    return lib, emu


def test_cpu_suite_under_host_sanitizers():
    rt = _asan_runtime()
    lib, emu = _build()
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, MOMFBD_LIBRARY=lib, MOMFBD_HOSTEMU=emu,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_library_cpu.py"),
                        os.path.join(ROOT, "tests", "test_hostemu_cpu.py")],
                       env=env, capture_output=True, text=True, cwd=ROOT, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "passed" in r.stdout
