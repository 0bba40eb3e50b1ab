"""Direct-encoding layout of a convolution's input and output ciphertexts
(oracle; test infrastructure only).

The paper packs zero-padded input channels into a ciphertext with direct
encoding (eq. de): data sit on the coefficients, c_n channels per ciphertext
(Algorithm 1, 'number of channel packing'), each channel's padded image in
row-major order; one output ciphertext per output channel. It leaves several
points open; this module fixes them as follows (the readings are listed in the
design notes):
  * c_n = floor(n / F) with F = (H + 2p)(W + 2p) the padded footprint, so the
    channel offset used by the second DRot of Algorithm 1 is (j mod c_n) * F;
  * a filter tap (ky, kx) is the shift ky * W' + kx in the padded image;
  * an input larger than n (F > n) is cut into row tiles with f_w - 1 halo
    rows, one ciphertext per (channel, tile), c_n = 1;
  * stride s > 1 with f_w > 1 computes the stride-1 grid and extracts every
    s-th row and column; for f_w = 1 the client encodes the subsampled input
    a[j][s y][s x] and the layer is a 1x1 stride-1 layer on that grid.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Plan:
    n: int
    c_i: int
    c_o: int
    h: int          # input height / width as given
    w: int
    f_w: int
    stride: int     # stride as given
    sub: int        # client-side subsampling factor (f_w == 1 and stride > 1), else 1
    s: int          # stride applied on the encoded grid (1 when sub > 1)
    he: int         # encoded input height / width (after client subsampling)
    we: int
    pad: int
    hp: int         # padded height / width
    wp: int
    F: int          # padded footprint hp * wp
    tiled: bool
    c_n: int        # channels per ciphertext
    T: int          # row tiles per channel
    r_o: int        # stride-1 output rows per tile
    G: int          # input ciphertexts
    G_w: int        # weight polynomials per output channel
    O: int          # output ciphertexts
    ho: int
    wo: int

    # -- positions --------------------------------------------------------
    def in_ct(self, j: int, tau: int) -> int:
        """Input ciphertext holding channel j, tile tau."""
        return (j // self.c_n) * self.T + tau

    def chan_off(self, j: int) -> int:
        """o_j: offset of channel j inside its ciphertext ((j mod c_n) * F; 0 when tiled)."""
        return (j % self.c_n) * self.F

    def tap_off(self, ky: int, kx: int) -> int:
        """s_k: shift of filter tap (ky, kx) in the padded row-major image."""
        return ky * self.wp + kx

    def weight_index(self, j: int) -> int:
        """Which weight polynomial W_{i, g_w} channel j contributes to."""
        return j if self.tiled else j // self.c_n

    def out_pos(self, oy: int, ox: int):
        """(tau, e): output pixel (oy, ox) sits at coefficient e of output ciphertext (i, tau)."""
        Y, X = self.s * oy, self.s * ox
        tau = Y // self.r_o
        return tau, (Y - tau * self.r_o) * self.wp + X

    def out_ct(self, i: int, tau: int) -> int:
        return i * self.T + tau


def plan(n: int, c_i: int, c_o: int, h: int, w: int, f_w: int, stride: int = 1) -> Plan:
    if f_w % 2 != 1 or f_w < 1:
        raise ValueError("filter width must be odd")
    if stride < 1:
        raise ValueError("stride must be positive")
    if f_w == 1 and stride > 1:
        sub, s = stride, 1
        he, we = -(-h // stride), -(-w // stride)
    else:
        sub, s = 1, stride
        he, we = h, w
    pad = (f_w - 1) // 2
    hp, wp = he + 2 * pad, we + 2 * pad
    F = hp * wp
    grid_rows = hp - f_w + 1                  # rows of the stride-1 output grid
    if F <= n:
        tiled, c_n, T, r_o = False, n // F, 1, grid_rows
        G = -(-c_i // c_n)
        G_w = G
    else:
        if f_w * wp > n:
            raise ValueError("padded row block does not fit one ciphertext")
        R = n // wp
        r_o = ((R - f_w + 1) // s) * s
        if r_o < 1:
            raise ValueError("no output row fits one ciphertext")
        tiled, c_n = True, 1
        T = -(-grid_rows // r_o)
        G, G_w = c_i * T, c_i
    ho = (hp - f_w) // s + 1
    wo = (wp - f_w) // s + 1
    return Plan(n, c_i, c_o, h, w, f_w, stride, sub, s, he, we, pad, hp, wp, F, tiled, c_n, T, r_o,
                G, G_w, c_o * T, ho, wo)


def encode_input(a, P: Plan) -> np.ndarray:
    """Direct encoding (eq. de) of one image a[c_i][h][w] (integers) into
    plaintext polynomials [G][n]: zero-padded channels, c_n per ciphertext,
    row tiles with halo when the padded image exceeds n."""
    a = np.asarray(a, dtype=np.int64)
    if P.sub > 1:
        a = a[:, :: P.sub, :: P.sub]
    assert a.shape == (P.c_i, P.he, P.we)
    m = np.zeros((P.G, P.n), dtype=np.int64)
    padded = np.zeros((P.c_i, P.hp, P.wp), dtype=np.int64)
    padded[:, P.pad:P.pad + P.he, P.pad:P.pad + P.we] = a
    rows_per_ct = P.r_o + P.f_w - 1 if P.tiled else P.hp
    for j in range(P.c_i):
        for tau in range(P.T):
            g = P.in_ct(j, tau)
            base = P.chan_off(j)
            y0 = tau * P.r_o
            for y in range(y0, min(y0 + rows_per_ct, P.hp)):
                k0 = base + (y - y0) * P.wp
                m[g, k0:k0 + P.wp] = padded[j, y]
    return m
