"""Conventional convolution with batch encoding: HRot (automorphism plus key
switching) and PMult (oracle; test infrastructure only).

Background: Homomorphic Encryption. Under batch encoding a plaintext
polynomial of R_t (t a prime = 1 mod 2n) holds n slots, its evaluations at the
roots of x^n + 1. HRot(ct, step) rotates the slots: the automorphism
x -> x^(3^step) is applied to both ciphertext polynomials, after which c1 is
under the key s(x^g); key switching returns it to s (eq. keySwitching): c1 is
split into digits of small coefficients (the decomposition with base 2^T),
each digit polynomial goes through the automorphism, and the switching keys
(swk0, swk1) of the step are multiplied in:
    c0' = c0(x^g) + sum_i swk0_i c1^(i)(x^g),   c1' = sum_i swk1_i c1^(i)(x^g).
PMult multiplies both polynomials by a plaintext polynomial.

Readings (the paper leaves these open):
  * slots form two rows of n/2 (the power-of-two cyclotomic's slot group is
    <3> x <-1>): slot (r, c) is the evaluation at psi^(e(r, c)) with
    e(0, c) = 3^c mod 2n and e(1, c) = -3^c mod 2n, psi the batch encoding's
    root (oracle.batch.slot_root). x -> x^(3^step) shifts both rows left by
    `step` (the paper's left-cyclic shift), x -> x^(-1) swaps the rows;
  * the decomposition: RNS limb l's residue split into D = ceil(30 / T)
    digits of T bits, digit (l, d) weighted by w_(l,d) = [q/q_l]
    [(q/q_l)^-1 mod q_l] 2^(T d), so that sum_(l,d) digit w = c1 (mod q);
  * the switching key of Galois element g for digit i = (l, d):
    swk0_i = -a_i s + e_i + w_i s(x^g), swk1_i = a_i (mod q), with a_i uniform
    and e_i a small error, both drawn by the caller;
  * the digits are taken of c1 before the automorphism (the paper's order:
    decompose, transform, automorphism, key switch), so one decomposition
    serves every rotation of a ciphertext.
Products are the schoolbook negacyclic product (the C form of oracle.ring's,
oracle.calg1.negacyclic_mul); no NTT.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from .batch import slot_root
from .calg1 import negacyclic_mul
from .params import centred, modulus


# ---------------------------------------------------------------- slots in rotation order
def slot_exponents(n: int) -> np.ndarray:
    """e[r][c]: the odd exponent of slot (r, c): 3^c mod 2n (row 0), -3^c mod 2n (row 1)."""
    m = 2 * n
    e = np.empty((2, n // 2), dtype=np.int64)
    v = 1
    for c in range(n // 2):
        e[0, c] = v
        e[1, c] = (m - v) % m
        v = (v * 3) % m
    return e


def _powers(w, n: int, t: int) -> np.ndarray:
    """M[k][j] = w_k^j mod t, j = 0 .. n-1."""
    w = np.asarray(w, dtype=np.int64)
    M = np.empty((len(w), n), dtype=np.int64)
    M[:, 0] = 1
    for j in range(1, n):
        M[:, j] = (M[:, j - 1] * w) % t
    return M


def rot_decode(p, t: int, n: int) -> np.ndarray:
    """Slots z[r][c] = p(psi^e(r, c)) mod t of a plaintext polynomial p."""
    p = np.asarray(p, dtype=np.int64) % t
    psi = slot_root(t, n)
    w = [pow(psi, int(ek), t) for ek in slot_exponents(n).reshape(-1)]
    M = _powers(w, n, t)
    return (((M * p[None, :]) % t).sum(axis=1) % t).reshape(2, n // 2)


def rot_encode(z, t: int, n: int) -> np.ndarray:
    """The polynomial p of degree < n with p(psi^e(r, c)) = z[r][c] (mod t):
    p_j = n^-1 sum over all slots of z psi^(-e j) (the slot exponents are all
    odd residues mod 2n, so sum_e psi^(e (i - j)) = n [i = j] for |i - j| < n)."""
    z = np.asarray(z, dtype=np.int64).reshape(-1) % t
    psi = slot_root(t, n)
    winv = [pow(psi, (2 * n - int(ek)) % (2 * n), t) for ek in slot_exponents(n).reshape(-1)]
    M = _powers(winv, n, t)
    s = ((M * z[:, None]) % t).sum(axis=0) % t
    return (s * pow(n, t - 2, t)) % t


# ---------------------------------------------------------------- automorphism, decomposition
def galois_element(step: int, swap: bool, n: int) -> int:
    """g = 3^step (x -1 when swap) mod 2n: x -> x^g rotates each slot row left
    by `step` and, with swap, exchanges the rows."""
    g = pow(3, step, 2 * n)
    return (2 * n - g) % (2 * n) if swap else g


def automorphism(a, g: int, q: int | None = None) -> np.ndarray:
    """a(x^g) mod (x^n + 1): coefficient j moves to j g mod 2n, negated when
    that lands in [n, 2n) (x^n = -1). g odd. Integer arrays of any sign; with
    q the result is reduced into [0, q)."""
    a = np.asarray(a, dtype=np.int64)
    n = a.shape[0]
    out = np.zeros(n, dtype=np.int64)
    for j in range(n):
        k = (j * g) % (2 * n)
        if k < n:
            out[k] += a[j]
        else:
            out[k - n] -= a[j]
    if q is not None:
        out %= q
    return out


def digit_count(T: int, bits: int = 30) -> int:
    return (bits + T - 1) // T


def decompose(c1, primes: Sequence[int], T: int) -> np.ndarray:
    """Digits of c1 [L][n] (residues): dig[l * D + d][j] = bits [T d, T d + T) of
    c1[l][j], values in [0, 2^T)."""
    c1 = np.asarray(c1, dtype=np.int64)
    L, n = c1.shape
    D = digit_count(T)
    dig = np.zeros((L * D, n), dtype=np.int64)
    for l in range(L):
        for d in range(D):
            dig[l * D + d] = (c1[l] >> (T * d)) & ((1 << T) - 1)
    return dig


def digit_weights(primes: Sequence[int], T: int) -> List[int]:
    """w_(l,d) = [q/q_l] [(q/q_l)^-1 mod q_l] 2^(T d) mod q, in digit order l * D + d."""
    q = modulus(primes)
    D = digit_count(T)
    out = []
    for ql in primes:
        Ml = q // ql
        base = Ml * pow(Ml, -1, ql)
        for d in range(D):
            out.append((base << (T * d)) % q)
    return out


def switching_key(s, g: int, a, e, primes: Sequence[int], T: int) -> np.ndarray:
    """Switching key of Galois element g: [L D][2][L][n] residues,
    key[i][0] = -a_i s + e_i + w_i s(x^g), key[i][1] = a_i.
    s: secret [n] (small integers); a: [L D][L][n] residues; e: [L D][n] small."""
    L = len(primes)
    n = len(s)
    w = digit_weights(primes, T)
    sg = automorphism(s, g)
    key = np.zeros((len(w), 2, L, n), dtype=np.int64)
    for i, wi in enumerate(w):
        for l, ql in enumerate(primes):
            ai = np.asarray(a[i][l], dtype=np.int64) % ql
            key[i, 0, l] = (-negacyclic_mul(ai, np.asarray(s) % ql, ql) + np.asarray(e[i]) + (wi % ql) * (sg % ql)) % ql
            key[i, 1, l] = ai
    return key.astype(np.uint32)


def hrot(ct, g: int, key, primes: Sequence[int], T: int) -> np.ndarray:
    """HRot by Galois element g with its switching key (see the module text):
    ct [2][L][n] residues -> [2][L][n]."""
    ct = np.asarray(ct, dtype=np.int64)
    L, n = ct.shape[1], ct.shape[2]
    dig = decompose(ct[1], primes, T)
    out = np.zeros((2, L, n), dtype=np.int64)
    for l, ql in enumerate(primes):
        out[0, l] = automorphism(ct[0, l], g, ql)
        for i in range(dig.shape[0]):
            di = automorphism(dig[i], g, ql)  # digit polynomial after the automorphism
            out[0, l] = (out[0, l] + negacyclic_mul(di, np.asarray(key[i][0][l], dtype=np.int64), ql)) % ql
            out[1, l] = (out[1, l] + negacyclic_mul(di, np.asarray(key[i][1][l], dtype=np.int64), ql)) % ql
    return out.astype(np.uint32)


def pmult(ct, p, primes: Sequence[int], t: int) -> np.ndarray:
    """PMult: both polynomials times the plaintext polynomial p (coefficients in
    [0, t) lifted to (-t/2, t/2]) in R_q, per limb."""
    ct = np.asarray(ct, dtype=np.int64)
    out = np.zeros_like(ct)
    for l, ql in enumerate(primes):
        pl = np.array([centred(int(v), t) % ql for v in p], dtype=np.int64)
        for c in range(2):
            out[c, l] = negacyclic_mul(ct[c, l], pl, ql)
    return out.astype(np.uint32)


# ---------------------------------------------------------------- the conventional convolution
class CLayout:
    """Slot layout of the conventional convolution (section "Conventional
    Convolution", its figure of the packed multi-channel convolution), read as
    follows (the paper gives the idea, not the index rules):
      * an image of h w <= n/2 pixels sits row-major in a block of bsz = (n/2)/c_r
        slots of one slot row; c_r = the largest power of two with c_r h w <= n/2
        channels per row, c_n = 2 c_r channels per ciphertext: channel
        j = g c_n + r c_r + k of input ciphertext g at row r, block k;
      * output ciphertexts use the same layout for the output channels;
      * stride 1, 'same' zero padding (f - 1)/2, cross-correlation;
      * rotations (swap, d, ky, kx): shift each row left by
        rho = (d bsz + (ky - p) w + (kx - p)) mod n/2, after exchanging the rows
        when swap: block (r, k) then holds input block (r xor swap, (k + d) mod c_r)
        moved by the tap offset, so one PMult with the right weights adds input
        channel j = g c_n + (r xor swap) c_r + (k + d) mod c_r, tap (ky, kx), to
        output channel o = o_g c_n + r c_r + k at every pixel;
      * out_(o_g) = sum_g sum_rotations PMult(HRot(in_g, rotation), pt(o_g, g, rotation)).
    A rotation with Galois element 1 (no swap, rho = 0) is the identity: no key switch."""

    def __init__(self, n: int, c_in: int, c_out: int, h: int, w: int, f: int):
        if f % 2 != 1:
            raise ValueError("odd filter width")
        hw = h * w
        if hw > n // 2:
            raise ValueError("the conventional layout here needs h w <= n/2")
        self.n, self.c_in, self.c_out, self.h, self.w, self.f = n, c_in, c_out, h, w, f
        self.p = (f - 1) // 2
        c_r = 1
        while 2 * c_r * hw <= n // 2:
            c_r *= 2
        self.c_r, self.bsz, self.c_n = c_r, (n // 2) // c_r, 2 * c_r
        self.G_in = -(-c_in // self.c_n)
        self.G_out = -(-c_out // self.c_n)
        self.rotations = []
        for swap in (0, 1):
            for d in range(c_r):
                for ky in range(f):
                    for kx in range(f):
                        rho = (d * self.bsz + (ky - self.p) * w + (kx - self.p)) % (n // 2)
                        self.rotations.append((swap, d, ky, kx, rho, galois_element(rho, bool(swap), n)))

    def encode_input(self, a, t: int) -> np.ndarray:
        """Slot vectors [G_in][2][n/2] of activations a [c_in][h][w] (values mod t)."""
        a = np.asarray(a, dtype=np.int64)
        z = np.zeros((self.G_in, 2, self.n // 2), dtype=np.int64)
        for j in range(self.c_in):
            g, rem = divmod(j, self.c_n)
            r, k = divmod(rem, self.c_r)
            z[g, r, k * self.bsz: k * self.bsz + self.h * self.w] = a[j].reshape(-1) % t
        return z

    def weight_slots(self, filters, o_g: int, g: int, rot: int, t: int) -> np.ndarray:
        """Slot vector [2][n/2] of the plaintext for output group o_g, input
        ciphertext g and rotation index rot (weights mod t, zero where the tap
        reads padding or a channel is absent)."""
        f = np.asarray(filters, dtype=np.int64)
        swap, d, ky, kx, _, _ = self.rotations[rot]
        z = np.zeros((2, self.n // 2), dtype=np.int64)
        for r in range(2):
            for k in range(self.c_r):
                o = o_g * self.c_n + r * self.c_r + k
                j = g * self.c_n + (r ^ swap) * self.c_r + (k + d) % self.c_r
                if o >= self.c_out or j >= self.c_in:
                    continue
                wv = int(f[o, j, ky, kx]) % t
                if wv == 0:
                    continue
                for y in range(self.h):
                    sy = y + ky - self.p
                    if not 0 <= sy < self.h:
                        continue
                    for x in range(self.w):
                        sx = x + kx - self.p
                        if 0 <= sx < self.w:
                            z[r, k * self.bsz + y * self.w + x] = wv
        return z

    def decode_output(self, z) -> np.ndarray:
        """Activations [c_out][h][w] from output slot vectors [G_out][2][n/2]."""
        z = np.asarray(z, dtype=np.int64)
        out = np.zeros((self.c_out, self.h, self.w), dtype=np.int64)
        for o in range(self.c_out):
            g, rem = divmod(o, self.c_n)
            r, k = divmod(rem, self.c_r)
            out[o] = z[g, r, k * self.bsz: k * self.bsz + self.h * self.w].reshape(self.h, self.w)
        return out


def conventional_conv(cts, filters, CL: CLayout, keys, primes: Sequence[int], t: int, T: int) -> np.ndarray:
    """out_(o_g) = sum_g sum_rot PMult(HRot(ct_g, rot), pt(o_g, g, rot)).
    cts: [G_in][2][L][n] residues (batch-encoded in the layout); keys[rot]: the
    switching key of rotation rot's Galois element (unused for the identity).
    Returns [G_out][2][L][n]."""
    L, n = len(primes), CL.n
    out = np.zeros((CL.G_out, 2, L, n), dtype=np.int64)
    qv = np.array(primes, dtype=np.int64)[None, :, None]
    for g in range(CL.G_in):
        for ri, (_, _, _, _, _, gal) in enumerate(CL.rotations):
            rc = np.asarray(cts[g], dtype=np.int64) if gal == 1 else hrot(cts[g], gal, keys[ri], primes, T)
            for o in range(CL.G_out):
                z = CL.weight_slots(filters, o, g, ri, t)
                if not z.any():
                    continue
                out[o] = (out[o] + pmult(rc, rot_encode(z, t, n), primes, t)) % qv
    return out.astype(np.uint32)
