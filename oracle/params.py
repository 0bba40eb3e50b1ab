"""Parameters of the ring and the plaintext encoding (oracle; test infrastructure only).

The paper works in R_q = Z_q[x]/(x^n + 1) with a single 60-bit q and plaintext
modulus p, Delta = floor(q / p) (Notation table, Background: Homomorphic
Encryption). This code uses an RNS modulus q = prod q_l of 30-bit primes with
q_l = 1 (mod 2n); by the CRT this is the same ring Z_q[x]/(x^n + 1). The
plaintext modulus is called t here (the paper's p) because p names the padding.
"""
from __future__ import annotations

from typing import List, Sequence


def is_prime_trial(m: int) -> bool:
    """Primality by trial division (plain and obviously correct for m < 2^32)."""
    if m < 2:
        return False
    if m % 2 == 0:
        return m == 2
    d = 3
    while d * d <= m:
        if m % d == 0:
            return False
        d += 2
    return True


def rns_primes(n: int, L: int, bits: int = 30) -> List[int]:
    """The L largest primes q < 2^bits with q = 1 (mod 2n), in descending order.

    q = 1 (mod 2n) makes Z_q contain a primitive 2n-th root of unity, which a
    negacyclic NTT needs; the oracle itself never uses an NTT.
    """
    out: List[int] = []
    step = 2 * n
    c = ((2 ** bits - 2) // step) * step + 1  # largest value < 2^bits that is 1 mod 2n
    while len(out) < L:
        if c < 2:
            raise ValueError("not enough primes")
        if is_prime_trial(c):
            out.append(c)
        c -= step
    return out


def modulus(primes: Sequence[int]) -> int:
    q = 1
    for ql in primes:
        q *= ql
    return q


def delta(q: int, t: int) -> int:
    """Delta = floor(q / t) (Notation table: floor(q/p))."""
    return q // t


def delta_limbs(primes: Sequence[int], t: int) -> List[int]:
    q = modulus(primes)
    d = delta(q, t)
    return [d % ql for ql in primes]


def centred(m: int, t: int) -> int:
    """Lift m in [0, t) to the representative in (-t/2, t/2] (plaintext coefficients
    of R_p lie in (-p/2, p/2], Background: Homomorphic Encryption)."""
    m %= t
    return m - t if 2 * m > t else m


def crt(residues: Sequence[int], primes: Sequence[int]) -> int:
    """The unique v in [0, q) with v = residues[l] (mod primes[l]) (Chinese remaindering)."""
    q = modulus(primes)
    v = 0
    for r, ql in zip(residues, primes):
        Ml = q // ql
        v += int(r) * Ml * pow(Ml, -1, ql)
    return v % q
