"""Server steps of the x^2 + x protocol on the GPU, through the C ABI: batch
encoding, PMult by 2r plus v (step 1) and the final combination (step 2),
bit-exact against oracle.batch; and the whole protocol at a ResNet-50 layer's
full size, every step on the GPU, against plain integer arithmetic."""
import numpy as np
import pytest

from oracle import batch, layout
from paper_2401_16732_amd import workloads as W

from gpu_util import dev, host, zeros

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_16732_amd import hconv
    hconv.load()
    return hconv


def _dev_i32(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).cuda()


@pytest.mark.parametrize("N,L,t", [(1024, 2, 12289), (2048, 1, 65537)])
def test_batch_encode_and_decode_match_oracle(hc, N, L, t):
    c = hc.Context(N, L, t)
    g = W.rng(N + t)
    z = g.integers(0, t, size=(3, N)).astype(np.uint32)
    z[0, :3] = [0, t - 1, t // 2]
    p = zeros((3, N))
    print(f"batch_encode N={N} t={t}", flush=True)
    c.batch_encode(dev(z), p)
    got = host(p)
    for k in range(3):
        assert (got[k] == batch.batch_encode(z[k], t, N)).all(), k
    q = g.integers(0, t, size=(2, N)).astype(np.uint32)
    zz = zeros((2, N))
    c.batch_decode(dev(q), zz)
    for k in range(2):
        assert (host(zz)[k] == batch.batch_decode(q[k], t, N)).all(), k


def test_batch_encoding_needs_a_prime_t(hc):
    c = hc.Context(1024, 2, 2 ** 17)
    with pytest.raises(hc.HcError) as err:
        c.batch_encode(zeros((1, 1024)), zeros((1, 1024)))
    assert err.value.status == -2
    with pytest.raises(hc.HcError):
        c.act_pmult(zeros((1, 2, 2, 1024)), zeros((1, 1024)), zeros((1, 1024)), zeros((1, 2, 2, 1024)),
                    zeros((c.act_workspace_words(1),)))


@pytest.mark.parametrize("N,L,t", [(1024, 3, 12289), (2048, 2, 65537)])
def test_act_pmult_matches_oracle(hc, N, L, t):
    c = hc.Context(N, L, t)
    g = W.rng(3 * N + L)
    n_ct = 2
    ct = W.gen_ct_limbs(g, (n_ct, 2), c.primes, N)
    r = g.integers(0, t, size=(n_ct, N)).astype(np.uint32)
    v = g.integers(0, t, size=(n_ct, N)).astype(np.uint32)
    exp = [batch.act_pmult(ct[k], r[k], v[k], c.primes, t, N) for k in range(n_ct)]
    ws = zeros((c.act_workspace_words(n_ct),))
    out = zeros((n_ct, 2, L, N))
    print(f"act_pmult N={N} L={L} t={t}", flush=True)
    c.act_pmult(dev(ct), dev(r), dev(v), out, ws)
    inplace = dev(ct)
    c.act_pmult(inplace, dev(r), dev(v), inplace, ws)
    for k in range(n_ct):
        assert (host(out)[k] == exp[k]).all(), k
        assert (host(inplace)[k] == exp[k]).all(), k


@pytest.mark.parametrize("N,L,t,shape", [
    (1024, 2, 12289, (30, 2, 9, 9, 3, 1)),
    (1024, 3, 65537, (2, 2, 40, 40, 3, 1)),      # row tiles
    (1024, 2, 2 ** 17, (6, 4, 15, 15, 1, 2)),    # subsampled; combine needs no batch encoding
])
def test_act_combine_matches_oracle(hc, N, L, t, shape):
    c = hc.Context(N, L, t)
    P = layout.plan(N, *shape)
    g = W.rng(11 * N + L)
    ly = hc.Layer(c, *shape, W.gen_filters(g, W.ConvSpec(*shape)))
    B = 2
    x = W.gen_ct_limbs(g, (B, P.G, 2), c.primes, N)
    y = W.gen_ct_limbs(g, (B, P.G, 2), c.primes, N)
    r = W.gen_mask(g, ly.act_shape(B), t)
    v = W.gen_mask(g, ly.act_shape(B), t)
    out = zeros(ly.in_shape(B))
    print(f"act_combine N={N} L={L} t={t} {shape}", flush=True)
    ly.act_combine(dev(x), dev(y), dev(r), dev(v), out, B)
    got = host(out)
    for b in range(B):
        rr = r[b].astype(np.int64)
        w = layout.encode_input((rr * rr - rr + v[b]) % t, P)
        for gi in range(P.G):
            assert (got[b, gi] == batch.act_combine(x[b, gi], y[b, gi], w[gi], c.primes, t)).all(), (b, gi)


def test_protocol_resnet50_layer_full_size(hc):
    """The x^2 + x protocol on the activation map entering ResNet-50's conv2_x
    3x3 layer (64 x 56 x 56) at N = 8192, 3 primes, t = 65537, every step on
    the GPU: batch-encrypted a + r, server step 1, decrypt + decode, direct
    re-encryption, server step 2, decryption. Result: a^2 + a mod t on every
    encoded coefficient."""
    N, L, t = 8192, 3, 65537
    shape = (64, 64, 56, 56, 3, 1)
    c = hc.Context(N, L, t)
    P = layout.plan(N, *shape)
    g = W.rng(65537)
    ly = hc.Layer(c, *shape, W.gen_filters(g, W.ConvSpec(*shape)))
    s = g.integers(-1, 2, size=N)
    sk = np.stack([np.mod(s, q) for q in c.primes]).astype(np.uint32)
    a, r, v = (W.gen_mask(g, ly.act_shape(1), t) for _ in range(3))
    u = (a.astype(np.int64) + r) % t
    n_slots = u.size
    n_ct = -(-n_slots // N)

    def slots(x):
        out = np.zeros(n_ct * N, dtype=np.uint32)
        out[:n_slots] = x.reshape(-1)
        return out.reshape(n_ct, N)

    def fresh_zero(n):
        ct = zeros((n, 2, L, N))
        c.encrypt_zero(dev(W.gen_ct_limbs(g, (n,), c.primes, N)), dev(sk),
                       _dev_i32(np.rint(g.normal(0, 3.2, size=(n, N))).clip(-19, 19)), ct,
                       zeros(((n + 1) * L * N,)))
        return ct

    print("protocol: client batch-encrypts a + r", flush=True)
    pu = zeros((n_ct, N))
    c.batch_encode(dev(slots(u)), pu)
    ct_b = fresh_zero(n_ct)
    c.encrypt_plain(pu, ct_b, ct_b)
    print("protocol: server step 1", flush=True)
    ct2 = zeros((n_ct, 2, L, N))
    c.act_pmult(ct_b, dev(slots(r)), dev(slots(v)), ct2, zeros((c.act_workspace_words(n_ct),)))
    print("protocol: client decrypts and decodes", flush=True)
    d = zeros((n_ct, N))
    c.decrypt(ct2, dev(sk), d, zeros(((n_ct + 1) * L * N,)))
    zz = zeros((n_ct, N))
    c.batch_decode(d, zz)
    z = host(zz).reshape(-1)[:n_slots].astype(np.int64)
    assert (z == (2 * r.reshape(-1).astype(np.int64) * u.reshape(-1) + v.reshape(-1)) % t).all()
    print("protocol: client re-encrypts under direct encoding; server step 2", flush=True)
    ct_x = fresh_zero(P.G)
    ly.encrypt_online(dev(((u * u + u) % t).astype(np.uint32)), ct_x, ct_x, 1)
    ct_y = fresh_zero(P.G)
    ly.encrypt_online(dev(z.reshape(ly.act_shape(1)).astype(np.uint32)), ct_y, ct_y, 1)
    ly.act_combine(ct_x, ct_y, dev(r), dev(v), ct_x, 1)
    m = zeros((P.G, N))
    c.decrypt(ct_x, dev(sk), m, zeros(((P.G + 1) * L * N,)))
    aa = a[0].astype(np.int64)
    assert (host(m) == layout.encode_input((aa * aa + aa) % t, P) % t).all()


def test_largest_ring_batch_encoding_properties(hc):
    """N = 16384 with t = 65537 (prime, 1 mod 2^15): decode(encode(z)) = z, and
    the slot-wise product equals the library's ring product modulo t (PMult's
    premise), on every slot. Properties that hold at any size; the oracle's
    O(N^2) interpolation is pinned at the smaller sizes."""
    N, L, t = 16384, 2, 65537
    c = hc.Context(N, L, t)
    ct_ = hc.Context(N, 1, t, primes=[t])   # the ring Z_t[x]/(x^N + 1) as a one-limb context
    g = W.rng(16385)
    z1 = g.integers(0, t, size=(1, N)).astype(np.uint32)
    z2 = g.integers(0, t, size=(1, N)).astype(np.uint32)
    p1, p2 = zeros((1, N)), zeros((1, N))
    c.batch_encode(dev(z1), p1)
    c.batch_encode(dev(z2), p2)
    back = zeros((1, N))
    c.batch_decode(p1, back)
    assert (host(back) == z1).all()
    prod = zeros((1, N))
    ct_.poly_mul(p1, p2, prod, zeros((2 * N,)))
    zz = zeros((1, N))
    c.batch_decode(prod, zz)
    assert (host(zz).astype(np.int64) == (z1.astype(np.int64) * z2) % t).all()


def test_client_and_protocol_steps_replay_as_graphs(hc):
    """The client and protocol entry points enqueue kernels and copies only, so
    they can be recorded in a HIP graph (as bench.py does to time them). Each
    replay, with eager work and synchronisations between replays, must give
    the eager result."""
    import torch
    N, L, t, B = 2048, 2, 65537, 2
    shape = (6, 5, 20, 20, 3, 1)
    c = hc.Context(N, L, t)
    g = W.rng(777)
    ly = hc.Layer(c, *shape, W.gen_filters(g, W.ConvSpec(*shape)))
    P = layout.plan(N, *shape)
    s = g.integers(-1, 2, size=N)
    sk = dev(np.stack([np.mod(s, q) for q in c.primes]).astype(np.uint32))
    act = dev(W.gen_mask(g, ly.act_shape(B), t))
    ct0 = dev(W.gen_ct_limbs(g, (B, P.G, 2), c.primes, N))
    c0 = dev(W.gen_ct_limbs(g, (B, P.c_o), c.primes, P.ho * P.wo))
    c1 = dev(W.gen_ct_limbs(g, (B, P.O), c.primes, N))
    n_ct = 3
    ctb = dev(W.gen_ct_limbs(g, (n_ct, 2), c.primes, N))
    r = dev(g.integers(0, t, size=(n_ct, N)).astype(np.uint32))
    v = dev(g.integers(0, t, size=(n_ct, N)).astype(np.uint32))
    enc, m, pm = zeros(ly.in_shape(B)), zeros(ly.mask_shape(B)), zeros((n_ct, 2, L, N))
    wsd, wsa = zeros((ly.decrypt_workspace_words(B),)), zeros((c.act_workspace_words(n_ct),))

    def work():
        ly.encrypt_online(act, ct0, enc, B)
        ly.decrypt_extracted(c0, c1, sk, m, B, wsd)
        c.act_pmult(ctb, r, v, pm, wsa)

    work()
    torch.cuda.synchronize()
    want = [host(x).copy() for x in (enc, m, pm)]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        work()
    for k in range(3):
        for x in (enc, m, pm):
            x.zero_()
        junk = torch.randint(0, 7, (1 << 20,), device="cuda", dtype=torch.int32).sum()  # eager work between
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for x, w_ in zip((enc, m, pm), want):
            assert (host(x) == w_).all(), k
        del junk
