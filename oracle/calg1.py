"""ctypes front of oracle/alg1.c (oracle; test infrastructure only).

build() compiles alg1.c with gcc into oracle/_alg1.so; load() builds it when
it is missing or older than its source.
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
_LIB = os.path.join(_HERE, "_alg1.so")
_lib = None


def build() -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", "-Wall", "-o", _LIB + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
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
    lib.oracle_alg1_points.restype = None
    lib.oracle_alg1_points.argtypes = [u32, u32, P, u32, u32, u32, P, P, P, P, P, ctypes.c_uint64,
                                       P, P, P, P, P, P]
    _lib = lib
    return lib


def threads() -> int:
    return int(load().oracle_threads())


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
