"""Pins for oracle.params and oracle.ring against mathematics and library routines."""
import json
import os

import numpy as np
import pytest
import sympy

from oracle import params, ring

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("n,L", [(4096, 2), (8192, 3), (16384, 4), (64, 3), (1024, 2)])
def test_rns_primes_are_the_largest_ntt_primes(n, L):
    ps = params.rns_primes(n, L)
    assert len(ps) == L and ps == sorted(ps, reverse=True)
    for q in ps:
        assert sympy.isprime(q) and q < 2 ** 30 and q % (2 * n) == 1
    # nothing larger than ps[0], and nothing between consecutive picks, qualifies
    grid = range(ps[-1], 2 ** 30, 2 * n)
    qualifying = [c for c in grid if sympy.isprime(c)]
    assert sorted(qualifying, reverse=True)[:L] == ps


def test_trial_division_agrees_with_sympy():
    g = np.random.Generator(np.random.PCG64(5))
    for m in list(range(0, 200)) + [int(v) for v in g.integers(2 ** 29, 2 ** 30, size=200)]:
        assert params.is_prime_trial(m) == sympy.isprime(m)


@pytest.mark.parametrize("t", [2 ** 17, 2 ** 20, 2 ** 24, 65537, 3])
def test_delta_is_the_floor(t):
    q = params.modulus(params.rns_primes(8192, 3))
    D = params.delta(q, t)
    assert D * t <= q < (D + 1) * t


def test_centred_lift():
    for t in (2 ** 17, 7, 8):
        for m in range(0, t, max(1, t // 97)):
            c = params.centred(m, t)
            assert -t / 2 < c <= t / 2 and (c - m) % t == 0


def test_crt_matches_sympy():
    ps = params.rns_primes(8192, 3)
    g = np.random.Generator(np.random.PCG64(6))
    for _ in range(50):
        res = [int(g.integers(0, q)) for q in ps]
        v = params.crt(res, ps)
        assert v == sympy.ntheory.modular.crt(ps, res)[0]
        assert all(v % q == r for q, r in zip(ps, res))


def _roots(n, q):
    """All roots of x^n + 1 in Z_q: the odd powers of a primitive 2n-th root of unity."""
    g = sympy.primitive_root(q)
    psi = pow(g, (q - 1) // (2 * n), q)
    assert pow(psi, n, q) == q - 1
    return [pow(psi, 2 * k + 1, q) for k in range(n)]


@pytest.mark.parametrize("n", [8, 32, 256])
def test_negacyclic_product_is_pointwise_at_roots(n):
    """Negacyclic convolution theorem: (a*b)(w) = a(w) b(w) at every root w of x^n + 1."""
    q = params.rns_primes(n, 1)[0]
    g = np.random.Generator(np.random.PCG64(n))
    a = g.integers(0, q, size=n)
    b = g.integers(0, q, size=n)
    c = ring.negacyclic_mul(a, b, q)
    ev = lambda p, w: sum(int(p[i]) * pow(w, i, q) for i in range(n)) % q
    for w in _roots(n, q)[:: max(1, n // 16)]:
        assert ev(c, w) == ev(a, w) * ev(b, w) % q


def test_negacyclic_product_matches_sympy_and_brute_force():
    n, q = 16, 97
    g = np.random.Generator(np.random.PCG64(3))
    x = sympy.symbols("x")
    for _ in range(10):
        a = g.integers(-50, 50, size=n)
        b = g.integers(-50, 50, size=n)
        pa = sympy.Poly(list(reversed([int(v) for v in a])), x)
        pb = sympy.Poly(list(reversed([int(v) for v in b])), x)
        r = sympy.rem(pa * pb, sympy.Poly(x ** n + 1, x))
        coeffs = list(reversed(r.all_coeffs()))
        coeffs += [0] * (n - len(coeffs))
        exact = ring.negacyclic_mul_small(a, b)
        assert [int(c) for c in coeffs] == exact
        assert list(ring.negacyclic_mul(a, b, q)) == [c % q for c in exact]


def test_x_to_the_n_is_minus_one():
    n, q = 16, 97
    xn1 = np.zeros(n, dtype=np.int64); xn1[n - 1] = 1
    x1 = np.zeros(n, dtype=np.int64); x1[1] = 1
    c = ring.negacyclic_mul(xn1, x1, q)
    assert c[0] == q - 1 and not c[1:].any()


def test_drot_golden_examples():
    with open(os.path.join(HERE, "golden", "drot_example.json")) as fh:
        cases = json.load(fh)["cases"]
    for cs in cases:
        assert list(ring.drot(np.array(cs["m"]), cs["step"])) == cs["expected"]


@pytest.mark.parametrize("step", [0, 1, 5, 31, 63])
def test_drot_is_multiplication_by_x_to_minus_step(step):
    n, q = 64, params.rns_primes(64, 1)[0]
    g = np.random.Generator(np.random.PCG64(step))
    c = g.integers(0, q, size=n)
    idx, sign = ring.monomial_inverse(step, n)
    mono = np.zeros(n, dtype=np.int64); mono[idx] = sign
    assert (ring.drot(c, step, q) == ring.negacyclic_mul(mono, c, q)).all()
    # and x^(-step) * x^step = 1
    fwd = np.zeros(n, dtype=np.int64); fwd[step] = 1
    one = ring.negacyclic_mul(mono % q, fwd, q)
    assert one[0] == 1 and not one[1:].any()
