"""Pins for the oracle's conventional convolution pieces (oracle/hrot.py):
slots in rotation order, the automorphism, the decomposition, key switching
(HRot) and the packed HRot/PMult convolution. Each is checked against what
the mathematics fixes, not against a retyping of itself:
  * the rotation-order slots are the batch encoding's slots (pinned in
    test_oracle_batch) in another order, and encoding inverts decoding;
  * x -> x^g is a ring homomorphism, composes multiplicatively, and shifts /
    swaps the slot rows as the paper's HRot states;
  * digits recombine to the residue, and weighted digits to c1 mod q (CRT);
  * HRot on a toy BFV ciphertext decrypts to the rotated message;
  * the conventional convolution decrypts to the plain convolution mod t
    (pinned to scipy elsewhere).
"""
import numpy as np
import pytest

from oracle import batch, bfv, calg1, conv, hrot, params, ring
from paper_2401_16732_amd import workloads as W


def _primes(n, L=3):
    return params.rns_primes(n, L)


@pytest.mark.parametrize("n,t", [(64, 257), (128, 257), (256, 7681)])
def test_slot_exponents_and_rotation_order_match_batch_slots(n, t):
    e = hrot.slot_exponents(n).reshape(-1)
    assert sorted(e.tolist()) == list(range(1, 2 * n, 2))  # every odd residue once
    g = W.rng(n)
    p = g.integers(0, t, size=n)
    zr = hrot.rot_decode(p, t, n)
    zb = batch.batch_decode(p, t, n)  # slot k at psi^(2 brv(k) + 1)
    bits = n.bit_length() - 1
    for r in range(2):
        for c in range(n // 2):
            k = batch.brv((int(hrot.slot_exponents(n)[r, c]) - 1) // 2, bits)
            assert zr[r, c] == zb[k]
    assert (hrot.rot_encode(zr, t, n) == p).all()
    z = g.integers(0, t, size=(2, n // 2))
    assert (hrot.rot_decode(hrot.rot_encode(z, t, n), t, n) == z).all()


@pytest.mark.parametrize("n", [16, 64, 1024])
def test_c_negacyclic_product_equals_schoolbook(n):
    """The C product the HRot oracle uses equals ring.negacyclic_mul (pinned to
    sympy and brute force elsewhere), also at the largest residues."""
    q = _primes(max(n, 64), 1)[0]
    g = W.rng(n + 7)
    a, b = g.integers(0, q, size=n), g.integers(0, q, size=n)
    a[0] = b[-1] = q - 1
    assert (calg1.negacyclic_mul(a, b, q) == ring.negacyclic_mul(a, b, q)).all()


@pytest.mark.parametrize("n", [64, 128])
def test_automorphism_is_a_ring_homomorphism_and_composes(n):
    q = _primes(n, 1)[0]
    g = W.rng(n + 1)
    a, b = g.integers(0, q, size=n), g.integers(0, q, size=n)
    for gal in (3, 5, 2 * n - 1, hrot.galois_element(7, True, n)):
        ab = ring.negacyclic_mul(a, b, q)
        assert (hrot.automorphism(ab, gal, q) == ring.negacyclic_mul(hrot.automorphism(a, gal, q),
                                                                     hrot.automorphism(b, gal, q), q)).all()
    assert (hrot.automorphism(hrot.automorphism(a, 3, q), 5, q) == hrot.automorphism(a, 15, q)).all()
    assert (hrot.automorphism(a, 1, q) == a % q).all()
    # x -> x^(2n-1) is x -> x^-1: x^1 maps to x^(2n-1) = -x^(n-1)
    e1 = np.zeros(n, dtype=np.int64)
    e1[1] = 1
    m = hrot.automorphism(e1, 2 * n - 1, q)
    assert m[n - 1] == q - 1 and m.sum() == q - 1


@pytest.mark.parametrize("n,t", [(64, 257), (128, 257)])
def test_automorphism_rotates_and_swaps_slot_rows(n, t):
    g = W.rng(n + 2)
    z = g.integers(0, t, size=(2, n // 2))
    p = hrot.rot_encode(z, t, n)
    for step in (0, 1, 5, n // 2 - 1):
        zs = hrot.rot_decode(hrot.automorphism(p, hrot.galois_element(step, False, n), t), t, n)
        assert (zs == np.roll(z, -step, axis=1)).all(), step  # left shift by step in each row
        zw = hrot.rot_decode(hrot.automorphism(p, hrot.galois_element(step, True, n), t), t, n)
        assert (zw == np.roll(z[::-1], -step, axis=1)).all(), step


def test_decomposition_recombines():
    n, T = 64, 10
    primes = _primes(n)
    g = W.rng(3)
    c1 = W.gen_ct_limbs(g, (1,), primes, n)[0]
    dig = hrot.decompose(c1, primes, T)
    D = hrot.digit_count(T)
    assert dig.min() >= 0 and dig.max() < 2 ** T
    for l in range(len(primes)):
        assert (sum(dig[l * D + d] << (T * d) for d in range(D)) == c1[l]).all()
    w = hrot.digit_weights(primes, T)
    q = params.modulus(primes)
    for j in range(0, n, 7):
        v = sum(int(dig[i, j]) * w[i] for i in range(len(w))) % q
        assert v == params.crt([int(c1[l, j]) for l in range(len(primes))], primes)


def _keys(g, s, gal, primes, T, n):
    LD = len(primes) * hrot.digit_count(T)
    a = np.stack([W.gen_ct_limbs(g, (1,), primes, n)[0] for _ in range(LD)])
    e = np.stack([bfv.sample_error(g, n) for _ in range(LD)])
    return hrot.switching_key(s, gal, a, e, primes, T)


@pytest.mark.parametrize("T", [6, 10])
def test_hrot_decrypts_to_the_rotated_message(T):
    n, t = 64, 257
    primes = _primes(n)
    g = W.rng(T)
    s = bfv.sample_secret(g, n)
    z = g.integers(0, t, size=(2, n // 2))
    m = hrot.rot_encode(z, t, n)
    mc = np.array([params.centred(int(v), t) for v in m])
    ct = bfv.encrypt_sk(mc, s, bfv.sample_a(g, primes, n), bfv.sample_error(g, n), primes, t)
    for step, swap in ((1, False), (3, True), (n // 2 - 2, False)):
        gal = hrot.galois_element(step, swap, n)
        out = hrot.hrot(ct, gal, _keys(g, s, gal, primes, T, n), primes, T)
        dec = np.array(bfv.decrypt(out, s, primes, t))
        want = np.roll(z[::-1] if swap else z, -step, axis=1)
        assert (hrot.rot_decode(dec, t, n) == want).all(), (step, swap)
    # a key made for another Galois element does not rotate correctly
    gal = hrot.galois_element(1, False, n)
    bad = hrot.hrot(ct, gal, _keys(g, s, hrot.galois_element(2, False, n), primes, T, n), primes, T)
    assert not (hrot.rot_decode(np.array(bfv.decrypt(bad, s, primes, t)), t, n) == np.roll(z, -1, axis=1)).all()


def test_pmult_multiplies_slots():
    n, t = 64, 257
    primes = _primes(n)
    g = W.rng(9)
    s = bfv.sample_secret(g, n)
    z, y = g.integers(0, t, size=(2, n // 2)), g.integers(0, t, size=(2, n // 2))
    mc = np.array([params.centred(int(v), t) for v in hrot.rot_encode(z, t, n)])
    ct = bfv.encrypt_sk(mc, s, bfv.sample_a(g, primes, n), bfv.sample_error(g, n), primes, t)
    out = hrot.pmult(ct, hrot.rot_encode(y, t, n), primes, t)
    assert (hrot.rot_decode(np.array(bfv.decrypt(out, s, primes, t)), t, n) == (z * y) % t).all()


CSHAPES = [  # (n, t, c_in, c_out, h, w, f)
    (64, 257, 3, 5, 4, 4, 3),     # c_r = 2: two channels per row, row swaps and block shifts
    (64, 257, 2, 2, 4, 8, 3),     # one channel per row (h w = n/2)
    (128, 257, 5, 3, 3, 5, 1),    # 1x1, c_r = 4, ragged channel groups
    (128, 257, 2, 3, 5, 5, 5),    # 5x5 taps
]


@pytest.mark.parametrize("shape", CSHAPES)
def test_conventional_conv_decrypts_to_plain_conv(shape):
    n, t, ci, co, h, w, f = shape
    T = 10
    primes = _primes(n)
    CL = hrot.CLayout(n, ci, co, h, w, f)
    g = W.rng(sum(shape))
    s = bfv.sample_secret(g, n)
    a = g.integers(0, t, size=(ci, h, w))
    filt = g.integers(-128, 128, size=(co, ci, f, f))
    zin = CL.encode_input(a, t)
    cts = []
    for k in range(CL.G_in):
        mc = np.array([params.centred(int(v), t) for v in hrot.rot_encode(zin[k], t, n)])
        cts.append(bfv.encrypt_sk(mc, s, bfv.sample_a(g, primes, n), bfv.sample_error(g, n), primes, t))
    keys = {ri: _keys(g, s, gal, primes, T, n) for ri, (*_, gal) in enumerate(CL.rotations) if gal != 1}
    out = hrot.conventional_conv(np.stack(cts), filt, CL, keys, primes, t, T)
    zout = np.stack([hrot.rot_decode(np.array(bfv.decrypt(out[o], s, primes, t)), t, n) for o in range(CL.G_out)])
    assert (CL.decode_output(zout) == conv.plain_conv_mod_t(a, filt, 1, t)).all()
