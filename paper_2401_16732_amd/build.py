"""Build libhconv.so (HIP, gfx950) in-tree.

    python -m paper_2401_16732_amd.build

Every source is compiled by hipcc for gfx950 only, one object per translation
unit, in parallel (the masked inverse NTT's template instances are split by
ring size over three objects), then linked into one shared library. Packed
FP32 instruction generation is disabled (-packed-fp32-ops: nothing here is
floating point, and the flag keeps the compiler from emitting those forms).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(HERE, "..", "include")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhconv.so")
SOURCES = [os.path.join(CSRC, f) for f in ("hc_host.cpp", "hc_server.cpp", "hc_client.cpp", "hc_ntt.hip",
                                           "hc_mac.hip", "hc_client.hip", "hc_direct.hip", "hc_intt_masked_small.hip",
                                           "hc_intt_masked_8k.hip", "hc_intt_masked_16k.hip", "hc_probe.hip",
                                           "hc_noalloc.hip", "hc_cconv.hip", "hc_cconv.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def kernel_sources() -> list:
    """Every file the device code is built from (sorted), for fingerprints."""
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.h")))


def kernel_fingerprint() -> str:
    """sha256[:16] over the names and contents of kernel_sources(): identifies
    the kernel code a profile was taken on."""
    import hashlib
    h = hashlib.sha256()
    for p in kernel_sources():
        h.update(os.path.basename(p).encode() + b"\0" + open(p, "rb").read())
    return h.hexdigest()[:16]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-I", INCLUDE, "-c", "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = max(1, min(len(SOURCES), os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libhconv.so")
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = glob.glob(os.path.join(CSRC, "*")) + [os.path.join(INCLUDE, "hc.h")]
    return any(os.path.getmtime(d) > t for d in deps)


if __name__ == "__main__":
    print(build(verbose=True))
