"""Build libhconv.so (HIP, gfx950) in-tree.

    python -m paper_2401_16732_amd.build

Every HIP source is compiled with hipcc for gfx950 only, with packed-FP32
instruction generation disabled (-packed-fp32-ops: nothing here is floating
point, and the flag keeps the compiler from emitting those forms at all).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhconv.so")
SOURCES = [os.path.join(CSRC, "hc_host.cpp"), os.path.join(CSRC, "hc_server.cpp"), os.path.join(CSRC, "hc_kernels.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(HERE, "..", "include"), "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libhconv.so")
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = SOURCES + [os.path.join(CSRC, "hc_internal.h"), os.path.join(CSRC, "hc_objects.h"),
                      os.path.join(HERE, "..", "include", "hc.h")]
    return any(os.path.getmtime(d) > t for d in deps)


if __name__ == "__main__":
    print(build(verbose=True))
