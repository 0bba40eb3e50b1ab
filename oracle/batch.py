"""Batch (SIMD) encoding and the server steps of the x^2 + x protocol (oracle;
test infrastructure only).

Section "Proposed Secure Computation of Polynomial Activation Function"
(and its figure of the 2PC protocol): after the masked convolution the client
holds a + r. It sends back [[a + r]] under batch encoding and
[[a^2 + 2ar + r^2 + a + r]] under direct encoding. The server
  1. multiplies [[a + r]] slot-wise by 2r (PMult, possible because of batch
     encoding) and hides the result with fresh random numbers v:
     [[2ar + 2r^2 + v]];
  2. once the client has returned that vector re-encrypted under direct
     encoding, combines [[a^2 + 2ar + r^2 + a + r]] - [[2ar + 2r^2 + v]] and
     the plaintext r^2 - r + v into [[a^2 + a]].
r, v and r^2 are drawn offline (section "Moving Data-independent Operations to
Offline Phase"); here they are inputs.

Batch encoding needs a prime plaintext modulus t = 1 (mod 2n). Z_t then holds
a primitive 2n-th root of unity psi, the n roots of x^n + 1 mod t are the odd
powers psi^(2i+1), and R_t = Z_t[x]/(x^n + 1) is isomorphic to Z_t^n by
evaluation at them (the slots). The paper fixes no slot order; this oracle
fixes one, which the GPU library follows as a public convention:
  * psi = the first x^((t-1)/(2n)), for x = 2, 3, ..., whose n-th power is -1;
  * slot k is the evaluation point psi^(2 brv(k) + 1), brv = bit reversal over
    log2(n) bits.
Encoding is interpolation at the slot points, written out as the inverse of
the evaluation map; no NTT is used.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .params import centred, delta, is_prime_trial, modulus
from .ring import negacyclic_mul


def brv(k: int, bits: int) -> int:
    return int(format(k, f"0{bits}b")[::-1], 2) if bits else 0


def slot_root(t: int, n: int) -> int:
    """psi: the first x^((t-1)/2n), x = 2, 3, ..., with psi^n = -1 mod t."""
    if not is_prime_trial(t) or (t - 1) % (2 * n):
        raise ValueError("batch encoding needs a prime t = 1 mod 2n")
    for x in range(2, t):
        c = pow(x, (t - 1) // (2 * n), t)
        if pow(c, n, t) == t - 1:
            return c
    raise ValueError("no primitive 2n-th root")


def slot_points(t: int, n: int) -> np.ndarray:
    """omega_k = psi^(2 brv(k) + 1), k = 0 .. n-1."""
    psi = slot_root(t, n)
    bits = n.bit_length() - 1
    return np.array([pow(psi, 2 * brv(k, bits) + 1, t) for k in range(n)], dtype=np.int64)


def _powers(w: np.ndarray, n: int, t: int) -> np.ndarray:
    """M[k][j] = w_k^j mod t, j = 0 .. n-1."""
    M = np.empty((len(w), n), dtype=np.int64)
    M[:, 0] = 1
    for j in range(1, n):
        M[:, j] = (M[:, j - 1] * w) % t
    return M


def batch_decode(p, t: int, n: int) -> np.ndarray:
    """Slots of the plaintext polynomial p: z_k = p(omega_k) mod t."""
    p = np.asarray(p, dtype=np.int64) % t
    M = _powers(slot_points(t, n), n, t)
    return ((M * p[None, :]) % t).sum(axis=1) % t


def batch_encode(z, t: int, n: int) -> np.ndarray:
    """The polynomial p of degree < n with p(omega_k) = z_k mod t for every slot:
    p_j = n^-1 sum_k z_k omega_k^(-j) (the evaluation points are the n distinct
    roots of x^n + 1, so sum_k omega_k^(i-j) = n [i = j] for |i - j| < n)."""
    z = np.asarray(z, dtype=np.int64) % t
    winv = np.array([pow(int(w), t - 2, t) for w in slot_points(t, n)], dtype=np.int64)
    M = _powers(winv, n, t)
    s = ((M * z[:, None]) % t).sum(axis=0) % t
    return (s * pow(n, t - 2, t)) % t


def _lift(p, t: int, ql: int) -> np.ndarray:
    """Plaintext coefficients in [0, t) as their centred values mod q_l."""
    return np.array([centred(int(v), t) % ql for v in p], dtype=np.int64)


def pmult(ct, p, primes: Sequence[int], t: int) -> np.ndarray:
    """PMult: both components times the plaintext polynomial p (centred lift),
    in R_q per limb. ct: [2][L][n] residues; returns [2][L][n] uint32."""
    ct = np.asarray(ct, dtype=np.int64)
    out = np.zeros_like(ct)
    for l, ql in enumerate(primes):
        pl = _lift(p, t, ql)
        for c in range(2):
            out[c, l] = negacyclic_mul(ct[c, l], pl, ql)
    return out.astype(np.uint32)


def add_plain(ct, p, primes: Sequence[int], t: int) -> np.ndarray:
    """[[m]] + p: c0 += Delta * (centred p) mod q_l (plaintext addition)."""
    D = delta(modulus(primes), t)
    out = np.asarray(ct, dtype=np.int64).copy()
    for l, ql in enumerate(primes):
        out[0, l] = (out[0, l] + (D % ql) * _lift(p, t, ql)) % ql
    return out.astype(np.uint32)


def act_pmult(ct_batch, r_slots, v_slots, primes: Sequence[int], t: int, n: int) -> np.ndarray:
    """Server step 1: [[2r (a + r) + v]] = PMult([[a + r]], encode(2r)) + encode(v),
    all under batch encoding. r_slots, v_slots: the slot values in [0, t)."""
    p2r = batch_encode((2 * np.asarray(r_slots, dtype=np.int64)) % t, t, n)
    pv = batch_encode(v_slots, t, n)
    return add_plain(pmult(ct_batch, p2r, primes, t), pv, primes, t)


def act_combine(ct_x, ct_y, w_poly, primes: Sequence[int], t: int) -> np.ndarray:
    """Server step 2: [[x]] - [[y]] + w under direct encoding, where x encrypts
    a^2 + 2ar + r^2 + a + r, y encrypts 2ar + 2r^2 + v and w(x) is the direct
    encoding of r^2 - r + v mod t; the result encrypts a^2 + a."""
    x = np.asarray(ct_x, dtype=np.int64)
    y = np.asarray(ct_y, dtype=np.int64)
    out = np.zeros_like(x)
    for l, ql in enumerate(primes):
        out[:, l] = (x[:, l] - y[:, l]) % ql
    return add_plain(out, w_poly, primes, t)
