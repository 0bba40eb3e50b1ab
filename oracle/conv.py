"""The paper's homomorphic convolution and its plaintext meaning (oracle; test
infrastructure only).

  alg1_conv       Algorithm 1 (Proposed convolution): CMult + DRot with lazy
                  int64 accumulation and one reduction per output (Employing
                  Lazy Reduction in Convolution).
  weight_poly     W_{i,g}(x) = sum_{j in g} sum_taps f[i][j][tap] x^(-(o_j + s_tap)):
                  Algorithm 1 for output channel i equals sum_g c_g * W_{i,g}
                  in R_q, because DRot is multiplication by x^(-step) (eq. drot)
                  and CMult by a scalar.
  plain_conv_mod_t  the cross-correlation the client recovers (mod t).
  mask_extract    the server mask HAdd([[a]], [[r]]) of the x^2+x protocol
                  (Proposed Secure Computation of Polynomial Activation
                  Function), taken as adding the trivial ciphertext
                  (Delta * r_centred, 0), then gathering the valid output
                  coefficients of c0; c1 is returned whole.
  freivalds_rhs   sum_g c_g * (sum_i rho_i W_{i,g}) for a random rho: equals
                  sum_i rho_i y_i, a full-size check at 1/c_o of the cost.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .layout import Plan
from .params import centred, delta, modulus
from .ring import drot, monomial_inverse, negacyclic_mul


def _taps(P: Plan):
    return [(ky, kx) for ky in range(P.f_w) for kx in range(P.f_w)]


def alg1_conv(x, filters, P: Plan, primes: Sequence[int], outputs=None) -> np.ndarray:
    """Algorithm 1 on one image.

    x: input ciphertexts [G][2][L][n] (residues); filters: int [c_o][c_i][f_w][f_w].
    outputs: optional list of output channels i (default all).
    Returns y [len(outputs) * T][2][L][n] in [0, q_l), output ciphertext (i, tau)
    at row (index of i in outputs) * T + tau.

    For output channel i and tile tau:
        partial = 0
        for each input channel j:
            c = x[ciphertext of (j, tau)]
            t = sum over taps k of DRot(c, s_k) * f[i][j][k]
            partial += DRot(t, o_j)          (o_j = (j mod c_n) * F)
        y = partial reduced mod q_l once
    """
    x = np.asarray(x, dtype=np.int64)
    f = np.asarray(filters, dtype=np.int64)
    outs = list(range(P.c_o)) if outputs is None else list(outputs)
    L = len(primes)
    y = np.zeros((len(outs) * P.T, 2, L, P.n), dtype=np.int64)
    taps = _taps(P)
    for oi, i in enumerate(outs):
        for tau in range(P.T):
            for p in range(2):
                for l in range(L):
                    partial = np.zeros(P.n, dtype=np.int64)
                    for j in range(P.c_i):
                        c = x[P.in_ct(j, tau), p, l]
                        t = np.zeros(P.n, dtype=np.int64)
                        for (ky, kx) in taps:
                            w = int(f[i, j, ky, kx])
                            if w:
                                t += drot(c, P.tap_off(ky, kx)) * w
                        partial += drot(t, P.chan_off(j))
                    y[oi * P.T + tau, p, l] = partial % primes[l]
    return y.astype(np.uint32)


def weight_poly(filters_i, P: Plan, g_w: int) -> np.ndarray:
    """W_{i,g_w}(x) as an integer polynomial (no modulus) for one output channel.

    filters_i: [c_i][f_w][f_w]. The taps of the channels mapped to g_w are
    placed at x^(-e), e = o_j + s_tap, using x^(-e) = -x^(n-e) for e > 0.
    """
    f = np.asarray(filters_i, dtype=np.int64)
    W = np.zeros(P.n, dtype=np.int64)
    for j in range(P.c_i):
        if P.weight_index(j) != g_w:
            continue
        for ky in range(P.f_w):
            for kx in range(P.f_w):
                e = P.chan_off(j) + P.tap_off(ky, kx)
                idx, sign = monomial_inverse(e, P.n)
                W[idx] += sign * int(f[j, ky, kx])
    return W


def ring_conv(x, filters, P: Plan, primes: Sequence[int], outputs=None) -> np.ndarray:
    """y_{i,tau} = sum_{g_w} c_{(g_w, tau)} * W_{i,g_w} by schoolbook products (slow; small n)."""
    x = np.asarray(x, dtype=np.int64)
    outs = list(range(P.c_o)) if outputs is None else list(outputs)
    L = len(primes)
    y = np.zeros((len(outs) * P.T, 2, L, P.n), dtype=np.int64)
    for oi, i in enumerate(outs):
        Ws = [weight_poly(filters[i], P, g) for g in range(P.G_w)]
        for tau in range(P.T):
            for g in range(P.G_w):
                ct = g * P.T + tau if P.tiled else g
                for p in range(2):
                    for l, ql in enumerate(primes):
                        y[oi * P.T + tau, p, l] = (y[oi * P.T + tau, p, l]
                                                   + negacyclic_mul(Ws[g] % ql, x[ct, p, l], ql)) % ql
    return y.astype(np.uint32)


def plain_conv_mod_t(a, filters, stride: int, t: int) -> np.ndarray:
    """z[i][oy][ox] = sum_j sum_{ky,kx} f[i][j][ky][kx] * a[j][s oy + ky - p][s ox + kx - p] mod t
    with zero padding p = (f_w - 1) / 2 ('same' padding; cross-correlation, the
    direction that DRot's left shift realises). Returns values in [0, t)."""
    a = np.asarray(a, dtype=np.int64)
    f = np.asarray(filters, dtype=np.int64)
    c_o, c_i, fw, _ = f.shape
    _, H, W = a.shape
    p = (fw - 1) // 2
    ap = np.zeros((c_i, H + 2 * p, W + 2 * p), dtype=np.int64)
    ap[:, p:p + H, p:p + W] = a
    ho = (H + 2 * p - fw) // stride + 1
    wo = (W + 2 * p - fw) // stride + 1
    z = np.zeros((c_o, ho, wo), dtype=np.int64)
    for ky in range(fw):
        for kx in range(fw):
            win = ap[:, ky: ky + stride * (ho - 1) + 1: stride, kx: kx + stride * (wo - 1) + 1: stride]
            z += np.einsum("ij,jyx->iyx", f[:, :, ky, kx], win)
    return z % t


def mask_extract(y, mask, P: Plan, primes: Sequence[int], t: int):
    """Share conversion and output extraction for one image.

    y: output ciphertexts [O][2][L][n]; mask: r[c_o][ho][wo] in [0, t).
    c0_ext[i][l][oy][ox] = c0_(i,tau)[e] + Delta_l * (r_centred mod q_l)  mod q_l
    c1_out[o][l][:]     = c1_o whole.
    """
    y = np.asarray(y, dtype=np.int64)
    q = modulus(primes)
    D = delta(q, t)
    L = len(primes)
    c0_ext = np.zeros((P.c_o, L, P.ho, P.wo), dtype=np.int64)
    for i in range(P.c_o):
        for oy in range(P.ho):
            for ox in range(P.wo):
                tau, e = P.out_pos(oy, ox)
                rb = centred(int(mask[i, oy, ox]), t)
                for l, ql in enumerate(primes):
                    c0_ext[i, l, oy, ox] = (int(y[P.out_ct(i, tau), 0, l, e]) + (D % ql) * (rb % ql)) % ql
    c1_out = y[:, 1].copy()
    return c0_ext.astype(np.uint32), c1_out.astype(np.uint32)


def freivalds_rhs(x, filters, rho, P: Plan, primes: Sequence[int]) -> np.ndarray:
    """sum_i rho_i y_i for one image, computed as sum_g c_g * W'_g with
    W'_g = sum_i rho_i W_{i,g}; rho[l][i] are residues mod q_l.

    The combined filter f'[j][tap] = sum_i rho_i f[i][j][tap] mod q_l is applied
    with Algorithm 1's DRot structure, reducing after every product because f'
    is no longer small. Returns [T][2][L][n].
    """
    x = np.asarray(x, dtype=np.int64)
    f = np.asarray(filters, dtype=np.int64)
    L = len(primes)
    out = np.zeros((P.T, 2, L, P.n), dtype=np.int64)
    taps = _taps(P)
    for l, ql in enumerate(primes):
        r = np.asarray(rho[l], dtype=np.int64) % ql
        fc = np.zeros((P.c_i, P.f_w, P.f_w), dtype=np.int64)
        for i in range(P.c_o):
            fc = (fc + r[i] * (f[i] % ql)) % ql
        for tau in range(P.T):
            for p in range(2):
                partial = np.zeros(P.n, dtype=np.int64)
                for j in range(P.c_i):
                    c = x[P.in_ct(j, tau), p, l]
                    tt = np.zeros(P.n, dtype=np.int64)
                    for (ky, kx) in taps:
                        tt = (tt + drot(c, P.tap_off(ky, kx), ql) * int(fc[j, ky, kx])) % ql
                    partial = (partial + drot(tt, P.chan_off(j), ql)) % ql
                out[tau, p, l] = partial
    return out


def freivalds_lhs(y, rho, P: Plan, primes: Sequence[int]) -> np.ndarray:
    """sum_i rho_i y_(i,tau) over output ciphertexts y [O][2][L][n]; returns [T][2][L][n]."""
    y = np.asarray(y, dtype=np.int64)
    L = len(primes)
    out = np.zeros((P.T, 2, L, P.n), dtype=np.int64)
    for l, ql in enumerate(primes):
        r = np.asarray(rho[l], dtype=np.int64) % ql
        for i in range(P.c_o):
            for tau in range(P.T):
                out[tau, :, l] = (out[tau, :, l] + r[i] * y[P.out_ct(i, tau), :, l]) % ql
    return out


def decrypt_extracted(c0_ext, c1_out, s, P: Plan, primes: Sequence[int], t: int) -> np.ndarray:
    """Client-side decryption of the extracted outputs (eq. bfv_dec): for output
    pixel (i, oy, ox) at coefficient e of ciphertext (i, tau), the phase is
    c0_ext[i][:, oy, ox] + (c1_(i,tau) * s)[e]; returns m[c_o][ho][wo] in [0, t)."""
    from .params import crt
    q = modulus(primes)
    L = len(primes)
    c1_out = np.asarray(c1_out, dtype=np.int64)
    m = np.zeros((P.c_o, P.ho, P.wo), dtype=np.int64)
    for i in range(P.c_o):
        c1s = {}
        for tau in range(P.T):
            o = P.out_ct(i, tau)
            c1s[tau] = [negacyclic_mul(s, c1_out[o, l], ql) for l, ql in enumerate(primes)]
        for oy in range(P.ho):
            for ox in range(P.wo):
                tau, e = P.out_pos(oy, ox)
                res = [(int(c0_ext[i, l, oy, ox]) + int(c1s[tau][l][e])) % primes[l] for l in range(L)]
                v = crt(res, primes)
                m[i, oy, ox] = ((t * v + q // 2) // q) % t
    return m


def mask_add(y_coeff: int, r: int, l: int, primes: Sequence[int], t: int) -> int:
    """One masked coefficient: y + Delta_l * (r_centred mod q_l) mod q_l (see mask_extract)."""
    ql = primes[l]
    D = delta(modulus(primes), t)
    return (int(y_coeff) + (D % ql) * (centred(int(r), t) % ql)) % ql
