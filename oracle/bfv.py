"""Toy secret-key BFV (oracle; test infrastructure only).

Follows the paper's Background: Homomorphic Encryption section:
  * private-key encryption (Table 2): c0 = [-(a s + e0) + Delta m]_q, c1 = a;
  * the decryption relation (eq. bfv_dec, Appendix A): Delta m + v = [c1 s + c0]_q,
    correct while ||v||_inf < Delta / 2;
  * Algorithm 2 (online encryption): [[m]] = [[0]] + Delta * m(x) with [[0]]
    precomputed offline (Moving Data-independent Operations to Offline Phase).
Plaintext coefficients are centred in (-t/2, t/2] (t is the paper's p).
Ciphertexts are stored per RNS limb: arrays [2][L][n] of residues in [0, q_l).
The random polynomials a, s, e are inputs, drawn by the caller.

The paper does not fix the secret or error distributions; the tests use a
uniform ternary s and a rounded Gaussian e (sigma 3.2, clipped at 6 sigma).
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .params import crt, delta, modulus
from .ring import negacyclic_mul


def sample_secret(g: np.random.Generator, n: int) -> np.ndarray:
    return g.integers(-1, 2, size=n, dtype=np.int64)


def sample_error(g: np.random.Generator, n: int, sigma: float = 3.2) -> np.ndarray:
    e = np.rint(g.normal(0.0, sigma, size=n)).astype(np.int64)
    bound = int(np.ceil(6 * sigma))
    return np.clip(e, -bound, bound)


def sample_a(g: np.random.Generator, primes: Sequence[int], n: int) -> np.ndarray:
    """Uniform a in R_q as residues [L][n] (uniform per limb = uniform mod q by CRT)."""
    return np.stack([g.integers(0, ql, size=n, dtype=np.int64) for ql in primes])


def encrypt_sk(m_centred, s, a, e, primes: Sequence[int], t: int) -> np.ndarray:
    """Private-key BFV encryption (Table 2): ([-(a s + e) + Delta m]_q, a).

    m_centred: plaintext coefficients in (-t/2, t/2] (direct encoding, eq. de);
    s, e: small integer polynomials; a: residues [L][n].
    Returns [2][L][n] uint32 residues.
    """
    q = modulus(primes)
    D = delta(q, t)
    m = np.asarray(m_centred, dtype=np.int64)
    n = m.shape[0]
    out = np.zeros((2, len(primes), n), dtype=np.int64)
    for l, ql in enumerate(primes):
        as_ = negacyclic_mul(a[l], s, ql)
        dm = ((D % ql) * (m % ql)) % ql
        out[0, l] = (-(as_ + np.asarray(e, dtype=np.int64)) + dm) % ql
        out[1, l] = np.asarray(a[l], dtype=np.int64) % ql
    return out.astype(np.uint32)


def encrypt_zero(s, a, e, primes: Sequence[int]) -> np.ndarray:
    """The offline ciphertext [[0]] = ([-(a s + e)]_q, a) (Algorithm 2's input)."""
    n = len(s)
    out = np.zeros((2, len(primes), n), dtype=np.int64)
    for l, ql in enumerate(primes):
        out[0, l] = (-(negacyclic_mul(a[l], s, ql) + np.asarray(e, dtype=np.int64))) % ql
        out[1, l] = np.asarray(a[l], dtype=np.int64) % ql
    return out.astype(np.uint32)


def online_encrypt(ct_zero, m_centred, primes: Sequence[int], t: int) -> np.ndarray:
    """Algorithm 2: [[m]] = [[0]] + Delta * m(x): only c0 changes."""
    q = modulus(primes)
    D = delta(q, t)
    m = np.asarray(m_centred, dtype=np.int64)
    out = np.asarray(ct_zero, dtype=np.int64).copy()
    for l, ql in enumerate(primes):
        out[0, l] = (out[0, l] + (D % ql) * (m % ql)) % ql
    return out.astype(np.uint32)


def phase(ct, s, primes: Sequence[int], positions=None) -> list:
    """[c1 s + c0]_q as integers in [0, q) (left side of eq. bfv_dec), via CRT.

    positions: optional coefficient indices to return (default: all).
    """
    ct = np.asarray(ct, dtype=np.int64)
    n = ct.shape[-1]
    pos = list(range(n)) if positions is None else [int(k) for k in positions]
    per_limb = []
    for l, ql in enumerate(primes):
        v = (negacyclic_mul(s, ct[1, l], ql) + ct[0, l]) % ql
        per_limb.append(v)
    return [crt([per_limb[l][k] for l in range(len(primes))], primes) for k in pos]


def decrypt(ct, s, primes: Sequence[int], t: int, positions=None) -> list:
    """BFV decryption: m = round(t * [c1 s + c0]_q / q) mod t, rounding half up.

    Returns plaintext coefficients in [0, t) at the requested positions.
    """
    q = modulus(primes)
    return [((t * v + q // 2) // q) % t for v in phase(ct, s, primes, positions)]


def noise_inf(ct, s, m_centred, primes: Sequence[int], t: int) -> int:
    """||v||_inf where v = [c1 s + c0 - Delta m]_q taken centred in (-q/2, q/2] (eq. bfv_dec)."""
    q = modulus(primes)
    D = delta(q, t)
    ph = phase(ct, s, primes)
    worst = 0
    for k, v in enumerate(ph):
        r = (v - D * int(m_centred[k])) % q
        if 2 * r > q:
            r -= q
        worst = max(worst, abs(r))
    return worst
