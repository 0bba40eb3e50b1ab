"""Arithmetic in R_q = Z_q[x]/(x^n + 1) (oracle; test infrastructure only).

Only definitions are used: the schoolbook negacyclic product and the closed
form of DRot proved in the paper's Appendix A (DRot with Direct Encoding).
"""
from __future__ import annotations

import numpy as np


def negacyclic_mul(a, b, q: int) -> np.ndarray:
    """Schoolbook product a(x) * b(x) mod (x^n + 1, q).

    c_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+n} a_i b_j  (x^n = -1), reduced to [0, q).
    Inputs are integer arrays of length n; q < 2^31 so every a_i * b_j (after
    reducing the inputs mod q) fits in int64, and the running sum is reduced
    after each row.
    """
    a = np.asarray(a, dtype=np.int64) % q
    b = np.asarray(b, dtype=np.int64) % q
    n = a.shape[0]
    assert b.shape[0] == n
    c = np.zeros(n, dtype=np.int64)
    for i in range(n):
        if a[i] == 0:
            continue
        row = (a[i] * b) % q          # a_i * b_j for j = 0..n-1
        c[i:] += row[: n - i]          # i + j < n: + x^(i+j)
        c[:i] -= row[n - i:]           # i + j >= n: x^(i+j) = -x^(i+j-n)
        c %= q
    return c


def negacyclic_mul_small(a, b) -> list:
    """Exact integer product a(x) * b(x) mod (x^n + 1) with no modulus (Python ints;
    for tiny rings and brute-force checks)."""
    n = len(a)
    c = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                c[k] += int(a[i]) * int(b[j])
            else:
                c[k - n] -= int(a[i]) * int(b[j])
    return c


def drot(c, step: int, q: int | None = None) -> np.ndarray:
    """DRot of one polynomial: c(x) * x^(-step) mod (x^n + 1)  (eq. drot).

    By the closed form in the Appendix A proof, coefficient i of the result is
    (-1)^floor((i + step) / n) * c[(i + step) mod n]: a left cyclic shift by
    `step` with the sign flipped on wrap-around. Works on int64 arrays of any
    magnitude (lazy sums) when q is None, else reduces into [0, q).
    Valid for 0 <= step < 2n.
    """
    c = np.asarray(c, dtype=np.int64)
    n = c.shape[0]
    idx = np.arange(n) + step
    sign = np.where((idx // n) % 2 == 1, -1, 1).astype(np.int64)
    out = sign * c[idx % n]
    if q is not None:
        out %= q
    return out


def monomial_inverse(e: int, n: int):
    """x^(-e) in R: returns (index, sign) with x^(-e) = sign * x^index.

    x^0 = 1 and, for 0 < e < n, x^(-e) = -x^(n - e) because x^n = -1
    (so x^(n-e) * x^e = x^n = -1).
    """
    if not 0 <= e < n:
        raise ValueError("exponent must lie in [0, n)")
    if e == 0:
        return 0, 1
    return n - e, -1
