"""Python binding of libhconv (include/hc.h): argument marshalling only.

Device buffers are torch tensors (dtype int32 holding the uint32 residues,
contiguous, on the library's HIP device); streams are torch.cuda streams.
Every step of the convolution runs in the library's HIP kernels; when the
library is missing this module raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhconv.so")

HC_OK = 0
_STATUS = {0: "HC_OK", -1: "HC_EINVAL", -2: "HC_EUNSUPPORTED", -3: "HC_ENOMEM", -4: "HC_EDEVICE", -5: "HC_ESTATE"}

SYMBOLS = [
    "hc_ctx_create", "hc_ctx_info", "hc_ctx_destroy", "hc_plan", "hc_layer_create", "hc_layer_destroy",
    "hc_layer_plan", "hc_workspace_size", "hc_conv", "hc_mask_extract", "hc_conv_masked", "hc_batch_create",
    "hc_batch_workspace_bytes", "hc_batch_run", "hc_batch_run_eager", "hc_batch_destroy", "hc_poly_mul",
    "hc_sync", "hc_status_string", "hc_last_error", "hc_plan_ring", "hc_ring_params",
    "hc_batch_run_timed", "hc_ctx_set_tuning", "hc_ctx_get_tuning",
    "hc_server_create", "hc_server_add_net", "hc_server_request_bytes", "hc_server_submit", "hc_server_step",
    "hc_server_poll", "hc_server_outputs", "hc_server_release", "hc_server_get_stats", "hc_server_sync",
    "hc_server_destroy", "hc_batch_autotune", "hc_layer_get_tuning", "hc_layer_clear_tuning",
    "hc_layer_get_tuning_for", "hc_valu_probe", "hc_conv_masked_noalloc", "hc_batch_run_pipelined",
    "hc_batch_get_mac_cap", "hc_batch_set_mac_cap",
    "hc_cconv_create", "hc_cconv_destroy", "hc_cconv_info", "hc_cconv_keys_size", "hc_cconv_keygen_workspace_size",
    "hc_cconv_keygen", "hc_cconv_workspace_size", "hc_cconv_run", "hc_rot_encode", "hc_rot_decode",
    "hc_check_residues", "hc_encrypt_online", "hc_decrypt_workspace_size", "hc_decrypt_extracted", "hc_decrypt",
    "hc_encrypt_zero", "hc_batch_encode", "hc_batch_decode", "hc_encrypt_plain", "hc_act_workspace_size",
    "hc_act_pmult", "hc_act_combine", "hc_conv_masked_direct",
]


class HcError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {_STATUS.get(status, status)} ({detail})")
        self.status = status


class ConvShape(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in ("c_in", "c_out", "h", "w", "f", "stride")]


class Tuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in ("fwd_elog", "inv_elog", "mac_rows", "mac_cols", "mac_row_groups",
                                               "mac_col_groups", "mac_depth", "mac_lds", "inv_polys", "mac_pre")]

    def as_tuple(self):
        return tuple(getattr(self, k) for k, _ in self._fields_)


class Layout(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in (
        "sub", "s", "h_enc", "w_enc", "pad", "h_pad", "w_pad", "footprint", "tiled", "cn", "tiles",
        "rows_out_per_tile", "in_cts", "w_cts", "out_cts", "ho", "wo")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load libhconv.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2401_16732_amd.build`")
    lib = ctypes.CDLL(path)
    P, u32, u64, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
    I = ctypes.c_int
    sig = {
        "hc_ctx_create": (I, [u32, u32, P, u64, I, P]),
        "hc_ctx_info": (I, [P, P, P]),
        "hc_ctx_destroy": (None, [P]),
        "hc_plan": (I, [P, P, P]),
        "hc_layer_create": (I, [P, P, P, P, P]),
        "hc_layer_destroy": (None, [P]),
        "hc_layer_plan": (I, [P, P]),
        "hc_workspace_size": (I, [P, u32, I, P]),
        "hc_conv": (I, [P, P, P, u32, P, sz, P]),
        "hc_mask_extract": (I, [P, P, P, P, P, u32, P]),
        "hc_conv_masked": (I, [P, P, P, P, P, u32, P, sz, P]),
        "hc_batch_create": (I, [P, P, u32, u32, P]),
        "hc_batch_workspace_bytes": (I, [P, P]),
        "hc_batch_run": (I, [P, P, P, P, P, P]),
        "hc_batch_run_eager": (I, [P, P, P, P, P, P]),
        "hc_batch_destroy": (None, [P]),
        "hc_poly_mul": (I, [P, P, P, P, u32, P, sz, P]),
        "hc_check_residues": (I, [P, P, sz, P, P]),
        "hc_encrypt_online": (I, [P, P, P, P, u32, P]),
        "hc_decrypt_workspace_size": (I, [P, u32, P]),
        "hc_decrypt_extracted": (I, [P, P, P, P, P, u32, P, sz, P]),
        "hc_decrypt": (I, [P, P, P, P, u32, P, sz, P]),
        "hc_encrypt_zero": (I, [P, P, P, P, P, u32, P, sz, P]),
        "hc_batch_encode": (I, [P, P, P, u32, P]),
        "hc_batch_decode": (I, [P, P, P, u32, P]),
        "hc_encrypt_plain": (I, [P, P, P, P, u32, P]),
        "hc_act_workspace_size": (I, [P, u32, P]),
        "hc_act_pmult": (I, [P, P, P, P, P, u32, P, sz, P]),
        "hc_act_combine": (I, [P, P, P, P, P, P, u32, P]),
        "hc_conv_masked_direct": (I, [P, P, P, P, P, u32, P]),
        "hc_sync": (I, [P]),
        "hc_status_string": (ctypes.c_char_p, [I]),
        "hc_last_error": (ctypes.c_char_p, []),
        "hc_plan_ring": (I, [u32, P, P]),
        "hc_ring_params": (I, [u32, u32, u64, P, P]),
        "hc_batch_run_timed": (I, [P, P, P, P, P, P, P]),
        "hc_ctx_set_tuning": (I, [P, P]),
        "hc_ctx_get_tuning": (I, [P, P]),
        "hc_server_create": (I, [P, P, P]),
        "hc_server_add_net": (I, [P, P, u32, P]),
        "hc_server_request_bytes": (I, [P, u32, P]),
        "hc_server_submit": (I, [P, u32, P, P, P]),
        "hc_server_step": (I, [P]),
        "hc_server_poll": (I, [P, P, u32, P]),
        "hc_server_outputs": (I, [P, ctypes.c_uint64, u32, P, P]),
        "hc_server_release": (I, [P, ctypes.c_uint64]),
        "hc_server_get_stats": (I, [P, P]),
        "hc_server_sync": (I, [P]),
        "hc_server_destroy": (None, [P]),
        "hc_batch_autotune": (I, [P, P, P, P, P, P, ctypes.c_char_p]),
        "hc_layer_get_tuning": (I, [P, P, P]),
        "hc_layer_clear_tuning": (I, [P]),
        "hc_layer_get_tuning_for": (I, [P, u32, P]),
        "hc_valu_probe": (I, [I, P]),
        "hc_conv_masked_noalloc": (I, [P, P, P, P, P, u32, P]),
        "hc_batch_run_pipelined": (I, [P, P, P, P, P, u64, u32, P]),
        "hc_batch_get_mac_cap": (I, [P, P]),
        "hc_batch_set_mac_cap": (I, [P, u32]),
        "hc_cconv_create": (I, [P, P, P, u32, P, P]),
        "hc_cconv_destroy": (None, [P]),
        "hc_cconv_info": (I, [P, P, P]),
        "hc_cconv_keys_size": (I, [P, P]),
        "hc_cconv_keygen_workspace_size": (I, [P, P]),
        "hc_cconv_keygen": (I, [P, P, P, P, P, P, sz, P]),
        "hc_cconv_workspace_size": (I, [P, u32, P]),
        "hc_cconv_run": (I, [P, P, P, P, u32, P, sz, P]),
        "hc_rot_encode": (I, [P, P, P, u32, P]),
        "hc_rot_decode": (I, [P, P, P, u32, P, sz, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != HC_OK:
        raise HcError(status, where, _lib.hc_last_error().decode())


def _dptr(t, name: str, device=None):
    """Device pointer of a contiguous int32 CUDA/HIP tensor."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous int32 device tensor")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name} is on device {t.device.index}, the context on {device}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def plan_ring(N, c_in, c_out, h, w, f, stride=1) -> Layout:
    """Layout of a convolution for ring degree N (host only)."""
    load()
    lay = Layout()
    sh = ConvShape(c_in, c_out, h, w, f, stride)
    _check(_lib.hc_plan_ring(N, ctypes.byref(sh), ctypes.byref(lay)), "hc_plan_ring")
    return lay


class ValuRates(ctypes.Structure):
    _fields_ = [("simple_ops_per_s", ctypes.c_double), ("mul_ops_per_s", ctypes.c_double),
                ("mad64_ops_per_s", ctypes.c_double), ("butterflies_per_s", ctypes.c_double),
                ("compute_units", ctypes.c_uint32), ("clock_hz", ctypes.c_double),
                ("measured_clock_hz", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def valu_probe(device: int = 0) -> dict:
    """Register-only VALU rates of the device (hc_valu_probe)."""
    load()
    r = ValuRates()
    _check(_lib.hc_valu_probe(device, ctypes.byref(r)), "hc_valu_probe")
    return r.as_dict()


def ring_params(N: int, L: int, t: int):
    """(primes, Delta mod q_l) that a context would use (host only)."""
    load()
    p = (ctypes.c_uint32 * L)()
    d = (ctypes.c_uint32 * L)()
    _check(_lib.hc_ring_params(N, L, t, p, d), "hc_ring_params")
    return list(p), list(d)


class Context:
    """RNS ring context: N, L primes (largest < 2^30 with q = 1 mod 2N unless
    given), plaintext modulus t; twiddle tables live on `device`."""

    def __init__(self, N: int, L: int, t: int, device: int = 0, primes: Optional[Sequence[int]] = None):
        lib = load()
        self.N, self.L, self.t, self.device = N, L, t, device
        h = ctypes.c_void_p()
        pr = None
        if primes is not None:
            self._pr = (ctypes.c_uint32 * L)(*primes)
            pr = ctypes.cast(self._pr, ctypes.c_void_p)
        _check(lib.hc_ctx_create(N, L, pr, t, device, ctypes.byref(h)), "hc_ctx_create")
        self.h = h
        p = (ctypes.c_uint32 * L)()
        d = (ctypes.c_uint32 * L)()
        _check(lib.hc_ctx_info(h, p, d), "hc_ctx_info")
        self.primes: List[int] = list(p)
        self.delta_mod_q: List[int] = list(d)

    def plan(self, c_in, c_out, h, w, f, stride=1) -> Layout:
        lay = Layout()
        sh = ConvShape(c_in, c_out, h, w, f, stride)
        _check(_lib.hc_plan(self.h, ctypes.byref(sh), ctypes.byref(lay)), "hc_plan")
        return lay

    def poly_mul(self, a, b, out, ws, stream=None):
        count = a.numel() // (self.L * self.N)
        if a.numel() != count * self.L * self.N or b.numel() != a.numel() or out.numel() < a.numel():
            raise ValueError("a, b, out must hold count * L * N words")
        if ws.numel() < 2 * a.numel():
            raise ValueError("ws must hold 2 * count * L * N words")
        _check(_lib.hc_poly_mul(self.h, _dptr(a, "a", self.device), _dptr(b, "b", self.device),
                                _dptr(out, "out", self.device), count, _dptr(ws, "ws", self.device),
                                ws.numel() * 4, _stream(stream)), "hc_poly_mul")

    def check_residues(self, polys, stream=None) -> int:
        """Number of words of `polys` (device int32 tensor, [..][L][N]) that are
        not below the prime of their limb."""
        npolys = polys.numel() // self.N
        if npolys * self.N != polys.numel() or npolys % self.L:
            raise ValueError("polys must hold a whole number of [L][N] blocks")
        n = ctypes.c_uint64()
        _check(_lib.hc_check_residues(self.h, _dptr(polys, "polys", self.device), npolys, _stream(stream),
                                      ctypes.byref(n)), "hc_check_residues")
        return n.value

    def encrypt_zero(self, a, sk, e, ct_zero, ws, stream=None):
        """ct_zero [count][2][L][N] <- (-(a s + e), a) for a [count][L][N] residues,
        sk [L][N] key residues and e [count][N] int32 errors (device tensors);
        ws: (count + 1) L N words."""
        ln = self.L * self.N
        count = a.numel() // ln
        if a.numel() != count * ln or sk.numel() != ln or e.numel() != count * self.N:
            raise ValueError("a must hold count * L * N words, sk L * N, e count * N")
        if ct_zero.numel() < 2 * count * ln or ws.numel() < (count + 1) * ln:
            raise ValueError("ct_zero must hold 2 * count * L * N words, ws (count + 1) * L * N")
        _check(_lib.hc_encrypt_zero(self.h, _dptr(a, "a", self.device), _dptr(sk, "sk", self.device),
                                    _dptr(e, "e", self.device), _dptr(ct_zero, "ct_zero", self.device), count,
                                    _dptr(ws, "ws", self.device), ws.numel() * 4, _stream(stream)),
               "hc_encrypt_zero")

    def _rows(self, t, name, per_row):
        n = t.numel() // per_row
        if n * per_row != t.numel():
            raise ValueError(f"{name} must hold a whole number of {per_row}-word rows")
        return n

    def batch_encode(self, z, p, stream=None):
        """p [n][N] <- plaintext polynomials whose slots are z [n][N] (t prime, = 1 mod 2N)."""
        n = self._rows(z, "z", self.N)
        if p.numel() < z.numel():
            raise ValueError("p must hold n * N words")
        _check(_lib.hc_batch_encode(self.h, _dptr(z, "z", self.device), _dptr(p, "p", self.device), n,
                                    _stream(stream)), "hc_batch_encode")

    def batch_decode(self, p, z, stream=None):
        n = self._rows(p, "p", self.N)
        if z.numel() < p.numel():
            raise ValueError("z must hold n * N words")
        _check(_lib.hc_batch_decode(self.h, _dptr(p, "p", self.device), _dptr(z, "z", self.device), n,
                                    _stream(stream)), "hc_batch_decode")

    def rot_encode(self, z, p, stream=None):
        """p [n][N] <- the plaintext polynomials whose slots in rotation order
        (two rows of N/2, row 0 first) are z [n][N] (values in [0, t))."""
        n = self._rows(z, "z", self.N)
        if p.numel() < n * self.N:
            raise ValueError("p must hold n * N words")
        _check(_lib.hc_rot_encode(self.h, _dptr(z, "z", self.device), _dptr(p, "p", self.device), n,
                                  _stream(stream)), "hc_rot_encode")

    def rot_decode(self, p, z, ws, stream=None):
        """z [n][N] <- the rotation-order slots of plaintext polynomials p [n][N]; ws: n N words."""
        n = self._rows(p, "p", self.N)
        if z.numel() < n * self.N or ws.numel() < n * self.N:
            raise ValueError("z and ws must hold n * N words")
        _check(_lib.hc_rot_decode(self.h, _dptr(p, "p", self.device), _dptr(z, "z", self.device), n,
                                  _dptr(ws, "ws", self.device), ws.numel() * 4, _stream(stream)), "hc_rot_decode")

    def encrypt_plain(self, p, ct_zero, ct, stream=None):
        """ct [n][2][L][N] <- ct_zero + Delta * p for plaintext polynomials p [n][N]."""
        n = self._rows(p, "p", self.N)
        if ct_zero.numel() < 2 * n * self.L * self.N or ct.numel() < 2 * n * self.L * self.N:
            raise ValueError("ct_zero and ct must hold n * 2 * L * N words")
        _check(_lib.hc_encrypt_plain(self.h, _dptr(p, "p", self.device), _dptr(ct_zero, "ct_zero", self.device),
                                     _dptr(ct, "ct", self.device), n, _stream(stream)), "hc_encrypt_plain")

    def act_workspace_words(self, n_ct: int) -> int:
        b = ctypes.c_size_t()
        _check(_lib.hc_act_workspace_size(self.h, n_ct, ctypes.byref(b)), "hc_act_workspace_size")
        return (b.value + 3) // 4

    def act_pmult(self, ct_batch, r, v, ct_out, ws, stream=None):
        """Server step 1 of the x^2 + x protocol: ct_out <- PMult(ct_batch, encode(2r)) + encode(v)."""
        n = self._rows(ct_batch, "ct_batch", 2 * self.L * self.N)
        if r.numel() != n * self.N or v.numel() != n * self.N or ct_out.numel() < ct_batch.numel():
            raise ValueError("r and v must hold n_ct * N slots, ct_out n_ct * 2 * L * N words")
        if ws.numel() < self.act_workspace_words(n):
            raise ValueError("ws too small (act_workspace_words)")
        _check(_lib.hc_act_pmult(self.h, _dptr(ct_batch, "ct_batch", self.device), _dptr(r, "r", self.device),
                                 _dptr(v, "v", self.device), _dptr(ct_out, "ct_out", self.device), n,
                                 _dptr(ws, "ws", self.device), ws.numel() * 4, _stream(stream)), "hc_act_pmult")

    def decrypt(self, ct, sk, m, ws, stream=None):
        """m [count][N] <- decryption of ct [count][2][L][N] under the key
        residues sk [L][N] (all device int32 tensors); ws: (count + 1) L N words."""
        ln = self.L * self.N
        count = ct.numel() // (2 * ln)
        if ct.numel() != count * 2 * ln or sk.numel() != ln or m.numel() < count * self.N:
            raise ValueError("ct must hold count * 2 * L * N words, sk L * N, m count * N")
        if ws.numel() < (count + 1) * ln:
            raise ValueError("ws must hold (count + 1) * L * N words")
        _check(_lib.hc_decrypt(self.h, _dptr(ct, "ct", self.device), _dptr(sk, "sk", self.device),
                               _dptr(m, "m", self.device), count, _dptr(ws, "ws", self.device), ws.numel() * 4,
                               _stream(stream)), "hc_decrypt")

    def sync(self):
        _check(_lib.hc_sync(self.h), "hc_sync")

    def set_tuning(self, fwd_elog=0, inv_elog=0, mac_rows=0, mac_cols=0, mac_row_groups=0, mac_col_groups=0,
                   mac_depth=0, mac_lds=0, inv_polys=0, mac_pre=0):
        t = Tuning(fwd_elog, inv_elog, mac_rows, mac_cols, mac_row_groups, mac_col_groups, mac_depth, mac_lds,
                   inv_polys, mac_pre)
        _check(_lib.hc_ctx_set_tuning(self.h, ctypes.byref(t)), "hc_ctx_set_tuning")

    def get_tuning(self):
        t = Tuning()
        _check(_lib.hc_ctx_get_tuning(self.h, ctypes.byref(t)), "hc_ctx_get_tuning")
        return t.as_tuple()

    def close(self):
        if getattr(self, "h", None):
            _lib.hc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Layer:
    """One convolution with its NTT-domain weights resident on the device
    (hc_layer_create: the offline weight encoding)."""

    def __init__(self, ctx: Context, c_in, c_out, h, w, f, stride, filters: np.ndarray, stream=None):
        filters = np.ascontiguousarray(filters, dtype=np.int8)
        if filters.shape != (c_out, c_in, f, f):
            raise ValueError("filters must be int8 [c_out][c_in][f][f]")
        self.ctx = ctx
        self.shape = (c_in, c_out, h, w, f, stride)
        sh = ConvShape(c_in, c_out, h, w, f, stride)
        hdl = ctypes.c_void_p()
        _check(_lib.hc_layer_create(ctx.h, ctypes.byref(sh), filters.ctypes.data_as(ctypes.c_void_p),
                                    _stream(stream), ctypes.byref(hdl)), "hc_layer_create")
        self.h = hdl
        lay = Layout()
        _check(_lib.hc_layer_plan(hdl, ctypes.byref(lay)), "hc_layer_plan")
        self.layout = lay

    def workspace_words(self, B: int, masked: bool) -> int:
        n = ctypes.c_size_t()
        _check(_lib.hc_workspace_size(self.h, B, 1 if masked else 0, ctypes.byref(n)), "hc_workspace_size")
        return (n.value + 3) // 4

    def _need(self, t, shape, name):
        n = 1
        for v in shape:
            n *= v
        if t.numel() < n:
            raise ValueError(f"{name} holds {t.numel()} words, the layout needs {n} ({tuple(shape)})")

    def conv(self, ct_in, ct_out, B: int, ws, stream=None):
        d = self.ctx.device
        self._need(ct_in, self.in_shape(B), "ct_in")
        self._need(ct_out, self.out_shape(B), "ct_out")
        self._need(ws, (self.workspace_words(B, False),), "ws")
        _check(_lib.hc_conv(self.h, _dptr(ct_in, "ct_in", d), _dptr(ct_out, "ct_out", d), B, _dptr(ws, "ws", d),
                            ws.numel() * 4, _stream(stream)), "hc_conv")

    def mask_extract(self, ct_out, mask, c0_ext, c1_out, B: int, stream=None):
        d = self.ctx.device
        self._need(ct_out, self.out_shape(B), "ct_out")
        self._need(mask, self.mask_shape(B), "mask")
        self._need(c0_ext, self.c0_shape(B), "c0_ext")
        self._need(c1_out, self.c1_shape(B), "c1_out")
        _check(_lib.hc_mask_extract(self.h, _dptr(ct_out, "ct_out", d), _dptr(mask, "mask", d),
                                    _dptr(c0_ext, "c0_ext", d), _dptr(c1_out, "c1_out", d), B, _stream(stream)),
               "hc_mask_extract")

    def conv_masked(self, ct_in, mask, c0_ext, c1_out, B: int, ws, stream=None):
        d = self.ctx.device
        self._need(ct_in, self.in_shape(B), "ct_in")
        self._need(mask, self.mask_shape(B), "mask")
        self._need(c0_ext, self.c0_shape(B), "c0_ext")
        self._need(c1_out, self.c1_shape(B), "c1_out")
        self._need(ws, (self.workspace_words(B, True),), "ws")
        _check(_lib.hc_conv_masked(self.h, _dptr(ct_in, "ct_in", d), _dptr(mask, "mask", d),
                                   _dptr(c0_ext, "c0_ext", d), _dptr(c1_out, "c1_out", d), B, _dptr(ws, "ws", d),
                                   ws.numel() * 4, _stream(stream)), "hc_conv_masked")

    def encrypt_online(self, act, ct_zero, ct_in, B: int, stream=None):
        """ct_in <- [[0]] + Delta * (direct encoding of act [B][c_in][h][w]);
        ct_in may be ct_zero itself (only c0 is then written)."""
        d = self.ctx.device
        self._need(act, self.act_shape(B), "act")
        self._need(ct_zero, self.in_shape(B), "ct_zero")
        self._need(ct_in, self.in_shape(B), "ct_in")
        _check(_lib.hc_encrypt_online(self.h, _dptr(act, "act", d), _dptr(ct_zero, "ct_zero", d),
                                      _dptr(ct_in, "ct_in", d), B, _stream(stream)), "hc_encrypt_online")

    def decrypt_workspace_words(self, B: int) -> int:
        n = ctypes.c_size_t()
        _check(_lib.hc_decrypt_workspace_size(self.h, B, ctypes.byref(n)), "hc_decrypt_workspace_size")
        return (n.value + 3) // 4

    def decrypt_extracted(self, c0_ext, c1_out, sk, m, B: int, ws, stream=None):
        """m [B][c_out][ho][wo] <- decryption of the masked conv's outputs under
        the key residues sk [L][N]."""
        d = self.ctx.device
        self._need(c0_ext, self.c0_shape(B), "c0_ext")
        self._need(c1_out, self.c1_shape(B), "c1_out")
        self._need(sk, (self.ctx.L, self.ctx.N), "sk")
        self._need(m, self.mask_shape(B), "m")
        self._need(ws, (self.decrypt_workspace_words(B),), "ws")
        _check(_lib.hc_decrypt_extracted(self.h, _dptr(c0_ext, "c0_ext", d), _dptr(c1_out, "c1_out", d),
                                         _dptr(sk, "sk", d), _dptr(m, "m", d), B, _dptr(ws, "ws", d),
                                         ws.numel() * 4, _stream(stream)), "hc_decrypt_extracted")

    def act_combine(self, ct_x, ct_y, r, v, ct_out, B: int, stream=None):
        """Server step 2 of the x^2 + x protocol for this layer's input:
        ct_out <- ct_x - ct_y + Delta * enc(r^2 - r + v)."""
        d = self.ctx.device
        for t_, name in ((ct_x, "ct_x"), (ct_y, "ct_y"), (ct_out, "ct_out")):
            self._need(t_, self.in_shape(B), name)
        self._need(r, self.act_shape(B), "r")
        self._need(v, self.act_shape(B), "v")
        _check(_lib.hc_act_combine(self.h, _dptr(ct_x, "ct_x", d), _dptr(ct_y, "ct_y", d), _dptr(r, "r", d),
                                   _dptr(v, "v", d), _dptr(ct_out, "ct_out", d), B, _stream(stream)),
               "hc_act_combine")

    NOALLOC_SCRATCH_BYTES = 128 << 20  # HC_NOALLOC_SCRATCH_BYTES

    def conv_masked_noalloc(self, ct_in, mask, c0_ext, c1_out, B: int, stream=None):
        """conv_masked without a workspace: the library's fixed per-device
        scratch array (NOALLOC_SCRATCH_BYTES) holds the intermediate values; no
        allocation. Calls that overlap on one device race."""
        d = self.ctx.device
        self._need(ct_in, self.in_shape(B), "ct_in")
        self._need(mask, self.mask_shape(B), "mask")
        self._need(c0_ext, self.c0_shape(B), "c0_ext")
        self._need(c1_out, self.c1_shape(B), "c1_out")
        _check(_lib.hc_conv_masked_noalloc(self.h, _dptr(ct_in, "ct_in", d), _dptr(mask, "mask", d),
                                           _dptr(c0_ext, "c0_ext", d), _dptr(c1_out, "c1_out", d), B,
                                           _stream(stream)), "hc_conv_masked_noalloc")

    def conv_masked_direct(self, ct_in, mask, c0_ext, c1_out, B: int, stream=None):
        """The same outputs as conv_masked, by the coefficient-domain convolution
        (Algorithm 1 as written; untiled layers)."""
        d = self.ctx.device
        self._need(ct_in, self.in_shape(B), "ct_in")
        self._need(mask, self.mask_shape(B), "mask")
        self._need(c0_ext, self.c0_shape(B), "c0_ext")
        self._need(c1_out, self.c1_shape(B), "c1_out")
        _check(_lib.hc_conv_masked_direct(self.h, _dptr(ct_in, "ct_in", d), _dptr(mask, "mask", d),
                                          _dptr(c0_ext, "c0_ext", d), _dptr(c1_out, "c1_out", d), B,
                                          _stream(stream)), "hc_conv_masked_direct")

    def tuning(self, B: Optional[int] = None):
        """(batch size, (fwd_elog, inv_elog, mac_rows, mac_cols, mac_row_groups, mac_col_groups, mac_depth,
        mac_lds, inv_polys, mac_pre)) of the set stored last, or of the set for B images when B is given;
        (0, (0, ...)) when there is none."""
        t = Tuning()
        if B is not None:
            st = _lib.hc_layer_get_tuning_for(self.h, B, ctypes.byref(t))
            if st == -5:
                return 0, t.as_tuple()
            _check(st, "hc_layer_get_tuning_for")
            return B, t.as_tuple()
        Bv = ctypes.c_uint32()
        _check(_lib.hc_layer_get_tuning(self.h, ctypes.byref(Bv), ctypes.byref(t)), "hc_layer_get_tuning")
        return Bv.value, t.as_tuple()

    def clear_tuning(self):
        _check(_lib.hc_layer_clear_tuning(self.h), "hc_layer_clear_tuning")

    # shapes of the device buffers for B images
    def act_shape(self, B):
        return (B, self.shape[0], self.shape[2], self.shape[3])

    def in_shape(self, B):
        return (B, self.layout.in_cts, 2, self.ctx.L, self.ctx.N)

    def out_shape(self, B):
        return (B, self.layout.out_cts, 2, self.ctx.L, self.ctx.N)

    def mask_shape(self, B):
        return (B, self.shape[1], self.layout.ho, self.layout.wo)

    def c0_shape(self, B):
        return (B, self.shape[1], self.ctx.L, self.layout.ho, self.layout.wo)

    def c1_shape(self, B):
        return (B, self.layout.out_cts, self.ctx.L, self.ctx.N)

    def close(self):
        if getattr(self, "h", None):
            _lib.hc_layer_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CConvLayout(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in ("c_r", "block", "c_n", "g_in", "g_out", "rotations",
                                               "decomp_bits", "digits")]


class CConv:
    """The conventional convolution (batch encoding, HRot with key switching,
    PMult; hc_cconv_*) of one layer, with its weight plaintexts resident on the
    device. Stride 1, h w <= N/2, a context whose t is a prime = 1 mod 2N."""

    def __init__(self, ctx: Context, c_in, c_out, h, w, f, filters: np.ndarray, decomp_bits: int = 10,
                 stream=None):
        load()
        self.ctx = ctx
        self.h = None
        f8 = np.ascontiguousarray(np.asarray(filters, dtype=np.int8))
        if f8.shape != (c_out, c_in, f, f):
            raise ValueError(f"filters must be [c_out][c_in][f][f] = {(c_out, c_in, f, f)}")
        sh = ConvShape(c_in, c_out, h, w, f, 1)
        h_ = ctypes.c_void_p()
        _check(_lib.hc_cconv_create(ctx.h, ctypes.byref(sh), f8.ctypes.data_as(ctypes.c_void_p), decomp_bits,
                                    _stream(stream), ctypes.byref(h_)), "hc_cconv_create")
        self.h = h_
        lay = CConvLayout()
        _check(_lib.hc_cconv_info(self.h, ctypes.byref(lay), None), "hc_cconv_info")
        gal = (ctypes.c_uint32 * lay.rotations)()
        _check(_lib.hc_cconv_info(self.h, ctypes.byref(lay), gal), "hc_cconv_info")
        self.layout = lay
        self.galois = list(gal)

    def _size(self, fn, *args):
        b = ctypes.c_size_t()
        _check(fn(self.h, *args, ctypes.byref(b)), fn.__name__)
        return (b.value + 3) // 4

    def keys_words(self) -> int:
        return self._size(_lib.hc_cconv_keys_size)

    def keygen_workspace_words(self) -> int:
        return self._size(_lib.hc_cconv_keygen_workspace_size)

    def workspace_words(self, B: int) -> int:
        return self._size(_lib.hc_cconv_workspace_size, B)

    def keygen(self, sk, a, e, keys, ws, stream=None):
        """Switching keys [rotations][digits][2][L][N] (NTT domain) from the key
        residues sk [L][N], uniform a [rotations][digits][L][N] and int32 errors
        e [rotations][digits][N]."""
        d, L, N = self.ctx.device, self.ctx.L, self.ctx.N
        R, LD = self.layout.rotations, self.layout.digits
        if sk.numel() != L * N or a.numel() != R * LD * L * N or e.numel() != R * LD * N:
            raise ValueError("sk [L][N], a [rotations][digits][L][N], e [rotations][digits][N]")
        if keys.numel() < self.keys_words() or ws.numel() < self.keygen_workspace_words():
            raise ValueError("keys or workspace too small")
        _check(_lib.hc_cconv_keygen(self.h, _dptr(sk, "sk", d), _dptr(a, "a", d), _dptr(e, "e", d),
                                    _dptr(keys, "keys", d), _dptr(ws, "ws", d), ws.numel() * 4, _stream(stream)),
               "hc_cconv_keygen")

    def run(self, keys, ct_in, ct_out, B: int, ws, stream=None):
        """ct_out [B][g_out][2][L][N] <- the convolution of ct_in [B][g_in][2][L][N]."""
        d, L, N = self.ctx.device, self.ctx.L, self.ctx.N
        if ct_in.numel() != B * self.layout.g_in * 2 * L * N or ct_out.numel() != B * self.layout.g_out * 2 * L * N:
            raise ValueError("ct_in [B][g_in][2][L][N], ct_out [B][g_out][2][L][N]")
        if keys.numel() < self.keys_words() or ws.numel() < self.workspace_words(B):
            raise ValueError("keys or workspace too small")
        _check(_lib.hc_cconv_run(self.h, _dptr(keys, "keys", d), _dptr(ct_in, "ct_in", d),
                                 _dptr(ct_out, "ct_out", d), B, _dptr(ws, "ws", d), ws.numel() * 4,
                                 _stream(stream)), "hc_cconv_run")

    def close(self):
        if self.h is not None and _lib is not None:
            _lib.hc_cconv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr_array(ts, name, device):
    arr = (ctypes.c_void_p * len(ts))()
    for k, t in enumerate(ts):
        arr[k] = _dptr(t, f"{name}[{k}]", device).value
    return arr


class Batch:
    """All layers of a network on B images, recorded once into a HIP graph
    (hc_batch_create / hc_batch_run)."""

    def __init__(self, ctx: Context, layers: Sequence[Layer], B: int):
        self.ctx, self.layers, self.B = ctx, list(layers), B
        arr = (ctypes.c_void_p * len(layers))(*[ly.h.value for ly in layers])
        h = ctypes.c_void_p()
        _check(_lib.hc_batch_create(ctx.h, arr, len(layers), B, ctypes.byref(h)), "hc_batch_create")
        self.h = h
        n = ctypes.c_size_t()
        _check(_lib.hc_batch_workspace_bytes(h, ctypes.byref(n)), "hc_batch_workspace_bytes")
        self.workspace_bytes = n.value

    def _args(self, ct_in, mask, c0, c1):
        d = self.ctx.device
        if not (len(ct_in) == len(mask) == len(c0) == len(c1) == len(self.layers)):
            raise ValueError("one buffer per layer is required")
        for k, ly in enumerate(self.layers):
            ly._need(ct_in[k], ly.in_shape(self.B), f"ct_in[{k}]")
            ly._need(mask[k], ly.mask_shape(self.B), f"mask[{k}]")
            ly._need(c0[k], ly.c0_shape(self.B), f"c0_ext[{k}]")
            ly._need(c1[k], ly.c1_shape(self.B), f"c1_out[{k}]")
        return (_ptr_array(ct_in, "ct_in", d), _ptr_array(mask, "mask", d), _ptr_array(c0, "c0_ext", d),
                _ptr_array(c1, "c1_out", d))

    def run(self, ct_in, mask, c0, c1, stream=None):
        self._keep = self._args(ct_in, mask, c0, c1)
        _check(_lib.hc_batch_run(self.h, *self._keep, _stream(stream)), "hc_batch_run")

    def run_eager(self, ct_in, mask, c0, c1, stream=None):
        a = self._args(ct_in, mask, c0, c1)
        _check(_lib.hc_batch_run_eager(self.h, *a, _stream(stream)), "hc_batch_run_eager")

    def run_pipelined(self, ct_in, mask, c0, c1, chunk_bytes=64 << 20, nbuf=3, stream=None):
        """The batch as a two-stream pipeline over output-channel chunks (eager)."""
        a = self._args(ct_in, mask, c0, c1)
        _check(_lib.hc_batch_run_pipelined(self.h, *a, int(chunk_bytes), int(nbuf), _stream(stream)),
               "hc_batch_run_pipelined")

    def autotune(self, ct_in, mask, c0, c1, cache_path=None, stream=None):
        """Pick each layer's launch shapes by timing every candidate on these buffers."""
        a = self._args(ct_in, mask, c0, c1)
        cp = None if cache_path is None else str(cache_path).encode()
        _check(_lib.hc_batch_autotune(self.h, *a, _stream(stream), cp), "hc_batch_autotune")

    @property
    def mac_cap(self):
        """Grid cap of the graph's DMA-staged MAC launches (0: none)."""
        v = ctypes.c_uint32()
        _check(_lib.hc_batch_get_mac_cap(self.h, ctypes.byref(v)), "hc_batch_get_mac_cap")
        return v.value

    @mac_cap.setter
    def mac_cap(self, cap):
        _check(_lib.hc_batch_set_mac_cap(self.h, int(cap)), "hc_batch_set_mac_cap")

    def run_timed(self, ct_in, mask, c0, c1, stream=None):
        """Eager run with HIP events around every kernel; returns milliseconds
        per stage: (forward NTT, multiply-accumulate, inverse NTT + mask + extract)."""
        a = self._args(ct_in, mask, c0, c1)
        ms = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
        _check(_lib.hc_batch_run_timed(self.h, *a, _stream(stream), ms), "hc_batch_run_timed")
        return tuple(ms)

    def close(self):
        if getattr(self, "h", None):
            _lib.hc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ServerConfig(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_uint64), ("max_batch", ctypes.c_uint32), ("streams", ctypes.c_uint32),
                ("max_inflight", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "admitted", "completed", "groups", "images", "queued",
                                               "arena_used", "arena_bytes", "direct_groups")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Server:
    """Continuous-batching request loop over resident layers (hc_server_*)."""

    def __init__(self, ctx: Context, arena_bytes: int, max_batch: int = 16, streams: int = 4, max_inflight: int = 0):
        self.ctx = ctx
        cfg = ServerConfig(arena_bytes, max_batch, streams, max_inflight)
        h = ctypes.c_void_p()
        _check(_lib.hc_server_create(ctx.h, ctypes.byref(cfg), ctypes.byref(h)), "hc_server_create")
        self.h = h
        self.nets = []

    def add_net(self, layers: Sequence[Layer]) -> int:
        arr = (ctypes.c_void_p * len(layers))(*[ly.h.value for ly in layers])
        nid = ctypes.c_uint32()
        _check(_lib.hc_server_add_net(self.h, arr, len(layers), ctypes.byref(nid)), "hc_server_add_net")
        self.nets.append(list(layers))
        return nid.value

    def request_bytes(self, net: int) -> int:
        n = ctypes.c_size_t()
        _check(_lib.hc_server_request_bytes(self.h, net, ctypes.byref(n)), "hc_server_request_bytes")
        return n.value

    def submit(self, net: int, ct_in, mask) -> int:
        """ct_in[k], mask[k]: layer k's inputs for one image (device tensors, B = 1 shapes);
        they must stay alive until the request completes."""
        layers = self.nets[net]
        if len(ct_in) != len(layers) or len(mask) != len(layers):
            raise ValueError("one input and one mask per layer")
        d = self.ctx.device
        for k, ly in enumerate(layers):
            ly._need(ct_in[k], ly.in_shape(1), f"ct_in[{k}]")
            ly._need(mask[k], ly.mask_shape(1), f"mask[{k}]")
        a = _ptr_array(ct_in, "ct_in", d)
        m = _ptr_array(mask, "mask", d)
        rid = ctypes.c_uint64()
        _check(_lib.hc_server_submit(self.h, net, a, m, ctypes.byref(rid)), "hc_server_submit")
        return rid.value

    def step(self):
        _check(_lib.hc_server_step(self.h), "hc_server_step")

    def poll(self, cap: int = 1024):
        ids = (ctypes.c_uint64 * cap)()
        n = ctypes.c_uint32()
        _check(_lib.hc_server_poll(self.h, ids, cap, ctypes.byref(n)), "hc_server_poll")
        return list(ids[: n.value])

    def outputs(self, rid: int, layer: int, net: int):
        """(c0_ext, c1_out) of a completed request's layer, copied to new device tensors."""
        import torch
        ly = self.nets[net][layer]
        c0p, c1p = ctypes.c_void_p(), ctypes.c_void_p()
        _check(_lib.hc_server_outputs(self.h, rid, layer, ctypes.byref(c0p), ctypes.byref(c1p)), "hc_server_outputs")
        c0 = torch.empty(ly.c0_shape(1)[1:], dtype=torch.int32, device=f"cuda:{self.ctx.device}")
        c1 = torch.empty(ly.c1_shape(1)[1:], dtype=torch.int32, device=f"cuda:{self.ctx.device}")
        _copy_from_ptr(c0, c0p.value)
        _copy_from_ptr(c1, c1p.value)
        return c0, c1

    def release(self, rid: int):
        _check(_lib.hc_server_release(self.h, rid), "hc_server_release")

    def stats(self):
        st = ServerStats()
        _check(_lib.hc_server_get_stats(self.h, ctypes.byref(st)), "hc_server_get_stats")
        return st.as_dict()

    def sync(self):
        _check(_lib.hc_server_sync(self.h), "hc_server_sync")

    def close(self):
        if getattr(self, "h", None):
            _lib.hc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _copy_from_ptr(dst, src_ptr: int):
    """Device-to-device copy of dst.numel() words from a raw device address (HIP runtime)."""
    import torch
    hip = _hip_runtime()
    torch.cuda.synchronize(dst.device)
    rc = hip.hipMemcpy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src_ptr), ctypes.c_size_t(dst.numel() * 4),
                       ctypes.c_int(3))  # hipMemcpyDeviceToDevice
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed: {rc}")


_hip = None


def _hip_runtime():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.restype = ctypes.c_int
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return _hip
