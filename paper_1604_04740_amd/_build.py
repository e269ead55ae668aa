"""Build the HIP library (libne.so) and its CPU self-test library for gfx950.

Every .hip file under csrc/ (except the self-test shim) is compiled with
hipcc into an object under _build/, then linked into libne.so next to this
file.  The self-test shim (host-side entry points over the same word
arithmetic) becomes libne_selftest.so, used only by the CPU tests.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libne.so")
SELFTEST_LIB = os.path.join(PKG, "libne_selftest.so")
SELFTEST_SRC = "ne_selftest_host.hip"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall",
         "-Wno-unused-result", "-I", INCLUDE, "-I", CSRC,
         # keep packed-fp32 instructions out of the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith(".hip") and f != SELFTEST_SRC)


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src[:-4] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(jobs: int = 8, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = _sources()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    tmp = SELFTEST_LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, *FLAGS, "-shared", "-o", tmp, os.path.join(CSRC, SELFTEST_SRC)],
                          stderr=subprocess.DEVNULL)
    os.replace(tmp, SELFTEST_LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
