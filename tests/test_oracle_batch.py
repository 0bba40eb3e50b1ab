"""Pins for the oracle's batch encoding and the x^2 + x protocol's server steps.

What fixes each function (none of these retypes the function under test):
  * slot points: they are n distinct roots of x^n + 1 mod t, i.e. all of them;
    the slots of p(x) = x are the slot points themselves;
  * encode/decode: inverse to each other both ways; a constant vector encodes
    to the constant polynomial; the slot-wise product is the ring product
    (schoolbook negacyclic product mod t), the property PMult relies on;
  * pmult/add_plain: act on decrypted, decoded slots as products and sums;
  * act_pmult/act_combine: the protocol run end to end with toy BFV gives
    2r(a + r) + v after the first step and a^2 + a after the second, computed
    in plain integers.
"""
import numpy as np
import pytest

from oracle import batch, bfv, params, ring
from paper_2401_16732_amd import workloads as W

CASES = [(8, 17), (64, 257), (64, 7681), (256, 65537)]


def _centred(p, t):
    p = np.asarray(p, dtype=np.int64) % t
    return np.where(2 * p > t, p - t, p)


@pytest.mark.parametrize("n,t", CASES)
def test_slot_points_are_all_roots_of_x_n_plus_1(n, t):
    w = batch.slot_points(t, n)
    assert len(set(int(v) for v in w)) == n
    assert all(pow(int(v), n, t) == t - 1 for v in w)
    assert (batch.batch_decode([0, 1] + [0] * (n - 2), t, n) == w).all()


@pytest.mark.parametrize("n,t", CASES)
def test_encode_and_decode_are_inverse(n, t):
    g = W.rng(n + t)
    z = g.integers(0, t, size=n)
    p = g.integers(0, t, size=n)
    assert (batch.batch_decode(batch.batch_encode(z, t, n), t, n) == z).all()
    assert (batch.batch_encode(batch.batch_decode(p, t, n), t, n) == p).all()
    c = int(g.integers(1, t))
    assert (batch.batch_encode([c] * n, t, n) == [c] + [0] * (n - 1)).all()


@pytest.mark.parametrize("n,t", CASES[:3])
def test_slotwise_product_is_the_ring_product(n, t):
    g = W.rng(3 * n + t)
    z1, z2 = g.integers(0, t, size=n), g.integers(0, t, size=n)
    lhs = ring.negacyclic_mul(batch.batch_encode(z1, t, n), batch.batch_encode(z2, t, n), t)
    assert (lhs == batch.batch_encode((z1 * z2) % t, t, n)).all()


def test_batch_encoding_rejects_unsuitable_t():
    with pytest.raises(ValueError):
        batch.slot_root(2 ** 17, 64)      # not prime
    with pytest.raises(ValueError):
        batch.slot_root(11, 64)           # prime, but not 1 mod 2n


def _enc(m_poly, s, g, primes, t, n):
    return bfv.encrypt_sk(_centred(m_poly, t), s, bfv.sample_a(g, primes, n), bfv.sample_error(g, n), primes, t)


@pytest.mark.parametrize("n,t", [(64, 257), (64, 7681)])
def test_pmult_and_add_plain_act_on_slots(n, t):
    primes = params.rns_primes(n, 2)
    g = W.rng(5 * n + t)
    s = bfv.sample_secret(g, n)
    z, w, u = (g.integers(0, t, size=n) for _ in range(3))
    ct = _enc(batch.batch_encode(z, t, n), s, g, primes, t, n)
    prod = batch.pmult(ct, batch.batch_encode(w, t, n), primes, t)
    assert (batch.batch_decode(bfv.decrypt(prod, s, primes, t), t, n) == (z * w) % t).all()
    summ = batch.add_plain(ct, batch.batch_encode(u, t, n), primes, t)
    assert (batch.batch_decode(bfv.decrypt(summ, s, primes, t), t, n) == (z + u) % t).all()


@pytest.mark.parametrize("n,t", [(64, 257), (256, 65537)])
def test_protocol_server_steps_give_a_squared_plus_a(n, t):
    """The figure's protocol with toy BFV. Direct encoding here puts value k on
    coefficient k (any layout gives the same arithmetic per coefficient)."""
    primes = params.rns_primes(n, 2)
    g = W.rng(7 * n + t)
    s = bfv.sample_secret(g, n)
    a, r, v = (g.integers(0, t, size=n) for _ in range(3))
    u = (a + r) % t                                          # client: a + r after decryption
    ct_batch = _enc(batch.batch_encode(u, t, n), s, g, primes, t, n)
    ct2 = batch.act_pmult(ct_batch, r, v, primes, t, n)      # server step 1
    z = batch.batch_decode(bfv.decrypt(ct2, s, primes, t), t, n)
    assert (z == (2 * r * u + v) % t).all()
    ct_y = _enc(z, s, g, primes, t, n)                       # client re-encrypts, direct encoding
    ct_x = _enc((u * u + u) % t, s, g, primes, t, n)
    w = (r * r - r + v) % t
    out = batch.act_combine(ct_x, ct_y, w, primes, t)        # server step 2
    assert (np.array(bfv.decrypt(out, s, primes, t)) == (a * a + a) % t).all()
