"""Build the native library in-tree: ``paper_1911_00093_amd/libhmat.so``.

HIP sources are compiled for gfx950 only; host-only C++ sources with g++.
Objects go to ``paper_1911_00093_amd/_build/``.  Usage:
``python -m paper_1911_00093_amd.build`` (or ``__graft_entry__.build()``).
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libhmat.so")

HIP_SOURCES = ["matvec.hip", "matvec_mr.hip", "krylov.hip", "inverse.hip", "krylov_batched.hip", "gmres.hip",
               "learned.hip", "diag.hip", "assemble_gpu.hip"]
HOST_SOURCES = ["pack.cpp", "assemble.cpp"]
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
INC = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
HIP_FLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-result"]
# host-only code: no fast-math, no FMA contraction (so the setup builder's
# floating-point results are reproducible across compilers)
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-pthread"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + p.stdout)
    return p.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    jobs = []
    objs = []
    for s in HIP_SOURCES:
        o = os.path.join(OUT, s + ".o")
        jobs.append([HIPCC] + HIP_FLAGS + INC + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in HOST_SOURCES:
        o = os.path.join(OUT, s + ".o")
        jobs.append(["g++"] + HOST_FLAGS + INC + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for out in ex.map(_run, jobs):
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs +
         ["-lpthread", "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"])
    os.replace(tmp, LIB)
    return LIB


# Host-only library with AddressSanitizer and UndefinedBehaviorSanitizer:
# the packer and the setup builder (pure host C++, no HIP), for CPU tests
# under the sanitizers (loaded with the ASan runtime preloaded).
SAN_LIB = os.path.join(OUT, "san", "libhmat_host_san.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
             "-fno-fast-math", "-Wall", "-pthread"]


def build_host_sanitized() -> str:
    os.makedirs(os.path.dirname(SAN_LIB), exist_ok=True)
    tmp = SAN_LIB + ".tmp%d" % os.getpid()
    _run(["g++"] + SAN_FLAGS + INC + [os.path.join(CSRC, s) for s in HOST_SOURCES] + ["-o", tmp])
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_host_sanitized())
    else:
        print(build(verbose="-v" in sys.argv))
