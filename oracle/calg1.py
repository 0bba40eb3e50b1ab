"""ctypes front of oracle/alg1.c (oracle; test infrastructure only).

build() compiles alg1.c with gcc (-O3 -march=native, OpenMP) into a shared
library named for the host CPU (oracle/_alg1_<cpu>.so, since -march=native code
only runs on the CPU it was built for); load() builds it when it is missing or
older than its source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence

import numpy as np

from .layout import Plan

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "alg1.c")
_lib = None


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or 'unknown'."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_key() -> str:
    import hashlib
    flags = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("flags"):
                flags = line
                break
    except OSError:
        pass
    return hashlib.sha256((cpu_model() + flags).encode()).hexdigest()[:12]


_LIB = os.path.join(_HERE, f"_alg1_{_cpu_key()}.so")


def build() -> str:
    tmp = f"{_LIB}.tmp{os.getpid()}"
    cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-shared", "-fPIC", "-std=gnu99", "-Wall", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    u32 = ctypes.c_uint32
    lib.oracle_alg1_layer.restype = ctypes.c_int
    lib.oracle_alg1_layer.argtypes = [u32, u32, P, u32, u32, u32, P, P, P, P, P, u32, P, P]
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_threads.argtypes = []
    lib.oracle_set_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_freivalds.restype = None
    lib.oracle_freivalds.argtypes = [u32, u32, P, u32, u32, u32, u32, P, P, P, P, P, P, P]
    lib.oracle_negacyclic_mul.restype = None
    lib.oracle_negacyclic_mul.argtypes = [u32, ctypes.c_uint64, P, P, P]
    lib.oracle_alg1_points.restype = None
    lib.oracle_alg1_points.argtypes = [u32, u32, P, u32, u32, u32, P, P, P, P, P, ctypes.c_uint64,
                                       P, P, P, P, P, P]
    _lib = lib
    return lib


def threads() -> int:
    return int(load().oracle_threads())


def set_threads(n: int) -> int:
    """Cap the OpenMP threads of the oracle's calls; returns the new count."""
    return int(load().oracle_set_threads(int(n)))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _layout_arrays(P: Plan):
    in_ct = np.array([P.in_ct(j, tau) for j in range(P.c_i) for tau in range(P.T)], dtype=np.uint32)
    chan = np.array([P.chan_off(j) for j in range(P.c_i)], dtype=np.uint32)
    taps = np.array([P.tap_off(ky, kx) for ky in range(P.f_w) for kx in range(P.f_w)], dtype=np.uint32)
    return in_ct, chan, taps


def alg1_layer(x, filters, P: Plan, primes: Sequence[int], outputs=None) -> np.ndarray:
    """Algorithm 1 for one image (C, OpenMP over outputs). Same contract as
    conv.alg1_conv: returns y [len(outputs) * T][2][L][n]."""
    lib = load()
    x = np.ascontiguousarray(x, dtype=np.uint32)
    assert x.shape == (P.G, 2, len(primes), P.n)
    f = np.ascontiguousarray(np.asarray(filters, dtype=np.int8).reshape(P.c_o, P.c_i, P.f_w * P.f_w))
    outs = np.arange(P.c_o, dtype=np.uint32) if outputs is None else np.asarray(outputs, dtype=np.uint32)
    q = np.asarray(primes, dtype=np.uint32)
    in_ct, chan, taps = _layout_arrays(P)
    y = np.empty((len(outs) * P.T, 2, len(primes), P.n), dtype=np.uint32)
    rc = lib.oracle_alg1_layer(P.n, len(primes), _ptr(q), P.c_i, P.T, len(taps), _ptr(taps), _ptr(chan),
                               _ptr(in_ct), _ptr(f), _ptr(x), len(outs), _ptr(outs), _ptr(y))
    if rc != 0:
        raise MemoryError("oracle_alg1_layer")
    return y


def alg1_points(x, filters, P: Plan, primes: Sequence[int], i, tau, p, l, m) -> np.ndarray:
    """Selected output coefficients y_(i,tau)[p][l][m] of Algorithm 1 (closed form)."""
    lib = load()
    x = np.ascontiguousarray(x, dtype=np.uint32)
    assert x.shape == (P.G, 2, len(primes), P.n)
    f = np.ascontiguousarray(np.asarray(filters, dtype=np.int8).reshape(P.c_o, P.c_i, P.f_w * P.f_w))
    q = np.asarray(primes, dtype=np.uint32)
    in_ct, chan, taps = _layout_arrays(P)
    cols = [np.ascontiguousarray(v, dtype=np.uint32) for v in (i, tau, p, l, m)]
    npts = cols[0].shape[0]
    val = np.empty(npts, dtype=np.uint32)
    lib.oracle_alg1_points(P.n, len(primes), _ptr(q), P.c_i, P.T, len(taps), _ptr(taps), _ptr(chan),
                           _ptr(in_ct), _ptr(f), _ptr(x), npts, *[_ptr(c) for c in cols], _ptr(val))
    return val


def freivalds_rhs(x, filters, rho, P: Plan, primes: Sequence[int]) -> np.ndarray:
    """sum_i rho_i y_(i,tau) of one image's Algorithm 1 outputs, by the closed
    form with the combined filter (C, OpenMP): same contract as
    conv.freivalds_rhs, rho[l][i] residues mod q_l; returns [T][2][L][n]."""
    lib = load()
    x = np.ascontiguousarray(x, dtype=np.uint32)
    assert x.shape == (P.G, 2, len(primes), P.n)
    f = np.ascontiguousarray(np.asarray(filters, dtype=np.int8).reshape(P.c_o, P.c_i, P.f_w * P.f_w))
    q = np.asarray(primes, dtype=np.uint32)
    r = np.ascontiguousarray(np.asarray(rho, dtype=np.uint64) % q[:, None].astype(np.uint64), dtype=np.uint32)
    assert r.shape == (len(primes), P.c_o)
    in_ct, chan, taps = _layout_arrays(P)
    z = np.empty((P.T, 2, len(primes), P.n), dtype=np.uint32)
    lib.oracle_freivalds(P.n, len(primes), _ptr(q), P.c_i, P.c_o, P.T, len(taps), _ptr(taps), _ptr(chan),
                         _ptr(in_ct), _ptr(f), _ptr(x), _ptr(r), _ptr(z))
    return z


def negacyclic_mul(a, b, q: int) -> np.ndarray:
    """Schoolbook a(x) b(x) mod (x^n + 1, q) (C, 128-bit sums): the same
    definition as ring.negacyclic_mul, faster for n in the thousands."""
    lib = load()
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int64) % q, dtype=np.uint64)
    b = np.ascontiguousarray(np.asarray(b, dtype=np.int64) % q, dtype=np.uint64)
    assert a.shape == b.shape and a.ndim == 1
    c = np.empty_like(a)
    lib.oracle_negacyclic_mul(a.shape[0], int(q), _ptr(a), _ptr(b), _ptr(c))
    return c.astype(np.int64)
