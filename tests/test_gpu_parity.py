"""GPU parity: every output of the HIP path equals the CPU oracle bit for bit.

The oracle is Algorithm 1 (C, int64 lazy accumulation) plus the mask/extract
definition; the NTT is checked through negacyclic products against the
schoolbook product. Inputs come from the seeded generators only.
"""
import numpy as np
import pytest

from oracle import bfv, calg1, conv, layout, params, ring
from paper_2401_16732_amd import workloads as W

from gpu_util import check_layer_points, dev, host, zeros

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_16732_amd import hconv
    hconv.load()
    return hconv


def _ctx(hc, N, L, t):
    c = hc.Context(N, L, t)
    assert c.primes == params.rns_primes(N, L)
    assert c.delta_mod_q == params.delta_limbs(c.primes, t)
    return c


@pytest.mark.parametrize("N", [1024, 2048, 4096, 8192, 16384])
def test_ntt_negacyclic_product(hc, N):
    print(f"poly_mul N={N}", flush=True)
    L = 2
    c = _ctx(hc, N, L, 2 ** 17)
    g = W.rng(N)
    count = 2
    a = W.gen_ct_limbs(g, (count,), c.primes, N)
    b = W.gen_ct_limbs(g, (count,), c.primes, N)
    # edge operands: the constant 1 and the monomial x^(N-1)
    a[1, 0] = 0
    a[1, 0, 0] = 1
    a[1, 1] = 0
    a[1, 1, N - 1] = 1
    out = zeros((count, L, N))
    ws = zeros((2 * count * L * N,))
    c.poly_mul(dev(a), dev(b), out, ws)
    got = host(out)
    for k in range(count):
        for l, q in enumerate(c.primes):
            assert (got[k, l] == ring.negacyclic_mul(a[k, l], b[k, l], q)).all(), (k, l)


SMALL = [  # (N, c_i, c_o, h, w, f, stride)
    (1024, 5, 3, 14, 14, 3, 1),     # c_n = 4, ragged second ciphertext
    (1024, 3, 4, 40, 40, 7, 2),     # tiled (F > N), stride 2, ragged last tile
    (1024, 6, 5, 20, 20, 1, 2),     # 1x1 stride 2: client subsampling
    (2048, 9, 2, 9, 9, 5, 1),       # f = 5, c_n = 11
    (2048, 1, 1, 30, 30, 3, 1),     # single channel
    (1024, 2, 3, 60, 30, 3, 1),     # tiled, stride 1
    (2048, 33, 7, 6, 6, 3, 2),      # many channels per ciphertext, stride 2
]


def _layer_case(hc, shape, B, seed):
    N, ci, co, h, w, fw, s = shape
    L, t = 2, 2 ** 17
    c = _ctx(hc, N, L, t)
    P = layout.plan(N, ci, co, h, w, fw, s)
    g = W.rng(seed)
    f = W.gen_filters(g, W.ConvSpec(ci, co, h, w, fw, s))
    x = W.gen_ct_limbs(g, (B, P.G, 2), c.primes, N)
    r = W.gen_mask(g, (B, co, P.ho, P.wo), t)
    ly = hc.Layer(c, ci, co, h, w, fw, s, f)
    assert (ly.layout.in_cts, ly.layout.out_cts, ly.layout.ho, ly.layout.wo) == (P.G, P.O, P.ho, P.wo)
    return c, P, f, x, r, ly


@pytest.mark.parametrize("shape", SMALL)
@pytest.mark.parametrize("B", [1, 3, 17])
def test_layer_bit_exact(hc, shape, B):
    print(f"layer {shape} B={B}", flush=True)
    c, P, f, x, r, ly = _layer_case(hc, shape, B, 1000 + B)
    dx, dr = dev(x), dev(r)
    # unfused: conv -> full ciphertexts; then mask + extract
    ct_out = zeros(ly.out_shape(B))
    ly.conv(dx, ct_out, B, zeros((ly.workspace_words(B, False),)))
    c0a, c1a = zeros(ly.c0_shape(B)), zeros(ly.c1_shape(B))
    ly.mask_extract(ct_out, dr, c0a, c1a, B)
    # fused
    c0b, c1b = zeros(ly.c0_shape(B)), zeros(ly.c1_shape(B))
    ly.conv_masked(dx, dr, c0b, c1b, B, zeros((ly.workspace_words(B, True),)))
    y_gpu = host(ct_out)
    c0a, c1a, c0b, c1b = host(c0a), host(c1a), host(c0b), host(c1b)
    for b in range(B):
        y = calg1.alg1_layer(x[b], f, P, c.primes)
        assert (y_gpu[b] == y).all(), f"image {b}: conv output differs"
        e0, e1 = conv.mask_extract(y, r[b], P, c.primes, c.t)
        assert (c0a[b] == e0).all() and (c1a[b] == e1).all(), f"image {b}: mask_extract differs"
    assert (c0b == c0a).all() and (c1b == c1a).all(), "fused path differs from unfused"


def test_config1_decrypt_invariant(hc):
    """Single layer, N=4096, 2 primes, t=2^17, 16->16, 16x16, 3x3: real toy-BFV
    encryptions; decrypt(HE-conv) - mask == plain conv mod t, and every output
    bit-exact against the oracle."""
    N, L, t = 4096, 2, 2 ** 17
    spec = W.ConvSpec(16, 16, 16, 16, 3, 1)
    c = _ctx(hc, N, L, t)
    P = layout.plan(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
    g = W.rng(2401)
    f = W.gen_filters(g, spec)
    a = W.gen_activations(g, spec, -128, 128)[0]
    sk = bfv.sample_secret(g, N)
    m = layout.encode_input(a, P)
    x = np.stack([bfv.encrypt_sk(m[k], sk, bfv.sample_a(g, c.primes, N), bfv.sample_error(g, N), c.primes, t)
                  for k in range(P.G)])[None]
    r = W.gen_mask(g, (1, spec.c_o, P.ho, P.wo), t)
    ly = hc.Layer(c, *[spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride], f)
    c0, c1 = zeros(ly.c0_shape(1)), zeros(ly.c1_shape(1))
    print("config1 conv_masked", flush=True)
    ly.conv_masked(dev(x), dev(r), c0, c1, 1, zeros((ly.workspace_words(1, True),)))
    c0, c1 = host(c0)[0], host(c1)[0]
    y = calg1.alg1_layer(x[0], f, P, c.primes)
    e0, e1 = conv.mask_extract(y, r[0], P, c.primes, t)
    assert (c0 == e0).all() and (c1 == e1).all()
    md = conv.decrypt_extracted(c0, c1, sk, P, c.primes, t)
    z = conv.plain_conv_mod_t(a, f, spec.stride, t)
    assert ((md.astype(np.int64) - r[0]) % t == z).all()


def test_resnet18_cifar_layers_sampled(hc):
    """ResNet-18/CIFAR conv stack at N=8192, 3 primes, t=2^20, one image, one
    launch sequence per layer: sampled outputs of every layer vs the oracle,
    plus a Freivalds check over all output channels of three layers."""
    N, L, t = 8192, 3, 2 ** 20
    c = _ctx(hc, N, L, t)
    g = W.rng(18)
    for k, spec in enumerate(W.resnet18_cifar()):
        print(f"r18-cifar layer {k} {spec}", flush=True)
        P = layout.plan(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
        f = W.gen_filters(g, spec)
        x = W.gen_ct_limbs(g, (1, P.G, 2), c.primes, N)
        r = W.gen_mask(g, (1, spec.c_o, P.ho, P.wo), t)
        ly = hc.Layer(c, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride, f)
        c0, c1 = zeros(ly.c0_shape(1)), zeros(ly.c1_shape(1))
        ly.conv_masked(dev(x), dev(r), c0, c1, 1, zeros((ly.workspace_words(1, True),)))
        check_layer_points(P, c.primes, t, x[0], f, r[0], host(c0)[0], host(c1)[0], g, npts=48)
        if k in (0, 7, 19):
            ct = zeros(ly.out_shape(1))
            ly.conv(dev(x), ct, 1, zeros((ly.workspace_words(1, False),)))
            rho = [g.integers(0, q, size=spec.c_o) for q in c.primes]
            lhs = conv.freivalds_lhs(host(ct)[0], rho, P, c.primes)
            rhs = conv.freivalds_rhs(x[0], f, rho, P, c.primes)
            assert (lhs == rhs).all(), f"Freivalds check failed on layer {k}"
        ly.close()


def test_error_paths(hc):
    c = _ctx(hc, 1024, 2, 2 ** 17)
    f = np.zeros((2, 2, 3, 3), dtype=np.int8)
    ly = hc.Layer(c, 2, 2, 8, 8, 3, 1, f)
    with pytest.raises(ValueError):
        ly.conv(zeros((1,)), zeros(ly.out_shape(1)), 1, zeros((ly.workspace_words(1, False),)))
    with pytest.raises(hc.HcError) as e:
        hc.Layer(c, 2, 2, 8, 8, 2, 1, np.zeros((2, 2, 2, 2), dtype=np.int8))
    assert e.value.status == -2
    with pytest.raises(hc.HcError) as e:
        hc.Context(1000, 2, 2 ** 17)
    assert e.value.status == -2
    with pytest.raises(hc.HcError) as e:
        hc.Context(1024, 1, 2 ** 17, primes=[1073692673 + 2])
    assert e.value.status == -1
    # B = 0 is a no-op
    ly.conv(zeros((1,)), zeros((1,)), 0, zeros((1,)))


# (images, channels per thread, image groups, channel groups, loads in flight, LDS-staged,
#  inverse NTT stages in the MAC epilogue)
MAC_VARIANTS = [(1, 8, 1, 4, 2, 0, 0), (1, 4, 1, 4, 2, 0, 0), (2, 4, 1, 4, 2, 0, 0), (4, 4, 1, 4, 2, 0, 0),
                (4, 2, 1, 4, 2, 0, 0), (8, 2, 1, 4, 2, 0, 0), (4, 4, 4, 2, 2, 0, 0), (4, 8, 4, 2, 2, 0, 0),
                (2, 8, 4, 2, 2, 0, 0), (4, 4, 2, 4, 2, 0, 0), (2, 4, 4, 4, 2, 0, 0), (1, 8, 2, 4, 2, 0, 0),
                (4, 8, 4, 2, 3, 0, 0), (2, 8, 4, 2, 4, 0, 0), (4, 4, 4, 2, 4, 0, 0), (4, 4, 2, 4, 4, 0, 0),
                (1, 8, 2, 4, 4, 0, 0), (2, 4, 4, 4, 4, 0, 0), (1, 8, 1, 4, 4, 0, 0), (4, 8, 4, 2, 2, 1, 0),
                (4, 8, 4, 2, 3, 1, 0), (4, 8, 2, 2, 2, 1, 0), (4, 8, 2, 2, 3, 1, 0), (2, 8, 4, 2, 3, 1, 0),
                (4, 4, 4, 2, 3, 1, 0), (2, 8, 2, 2, 3, 1, 0), (4, 8, 4, 2, 2, 1, 5), (4, 8, 2, 2, 2, 1, 5),
                (4, 8, 2, 2, 3, 1, 5), (4, 8, 2, 2, 3, 2, 0), (4, 8, 2, 2, 4, 2, 0), (4, 8, 2, 2, 6, 2, 0),
                (4, 8, 4, 2, 3, 2, 0), (4, 8, 4, 2, 4, 2, 0), (2, 8, 4, 2, 4, 2, 0), (4, 4, 4, 2, 4, 2, 0),
                (2, 8, 2, 2, 4, 2, 0), (4, 4, 2, 2, 4, 2, 0), (4, 8, 2, 2, 3, 2, 5), (4, 8, 2, 2, 4, 2, 5),
                (4, 8, 4, 2, 4, 2, 5), (4, 8, 2, 2, 3, 2, 6), (4, 8, 2, 2, 4, 2, 6), (4, 8, 4, 2, 3, 2, 6),
                (4, 8, 4, 2, 4, 2, 6)]


def mac_tuning(v, inv_elog=0, inv_polys=0):
    """set_tuning arguments for MAC variant v (and optional inverse-NTT shape)."""
    return (0, inv_elog, *v[:6], inv_polys, v[6])


@pytest.mark.parametrize("N,elogs", [(8192, (3, 4, 5)), (16384, (4, 5)), (4096, (3, 4, 5)), (1024, (3, 4))])
def test_every_launch_shape_gives_the_same_bits(hc, N, elogs):
    """Autotuner candidates: every NTT thread shape and MAC tile produces the oracle's bits."""
    L, t, B = 2, 2 ** 17, 3
    c = _ctx(hc, N, L, t)
    spec = W.ConvSpec(20, 13, 12, 12, 3, 1)
    P = layout.plan(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
    g = W.rng(N + 5)
    f = W.gen_filters(g, spec)
    x = W.gen_ct_limbs(g, (B, P.G, 2), c.primes, N)
    r = W.gen_mask(g, (B, spec.c_o, P.ho, P.wo), t)
    ly = hc.Layer(c, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride, f)
    exp = [conv.mask_extract(calg1.alg1_layer(x[b], f, P, c.primes), r[b], P, c.primes, t) for b in range(B)]
    dx, dr = dev(x), dev(r)
    ws = zeros((ly.workspace_words(B, True),))
    cases = [(fe, ie, 0, 0, 0, 0) for fe in elogs for ie in elogs]
    cases += [mac_tuning(v) for v in MAC_VARIANTS if N >= 4096 or v[6] == 0]
    # two inverse-NTT polynomials per workgroup; B * out_cts = 39 leaves the last pair half empty
    cases += [(0, ie, 0, 0, 0, 0, 0, 0, 2) for ie in elogs if ie <= 4]
    for tune in cases:
        print(f"N={N} tuning {tune}", flush=True)
        c.set_tuning(*tune)
        c0, c1 = zeros(ly.c0_shape(B)), zeros(ly.c1_shape(B))
        ly.conv_masked(dx, dr, c0, c1, B, ws)
        c0, c1 = host(c0), host(c1)
        for b in range(B):
            assert (c0[b] == exp[b][0]).all() and (c1[b] == exp[b][1]).all(), (tune, b)
    with pytest.raises(hc.HcError):
        c.set_tuning(7, 0, 0, 0)
    with pytest.raises(hc.HcError):
        c.set_tuning(0, 0, 3, 3, 1, 1)
    with pytest.raises(hc.HcError):
        c.set_tuning(0, 0, 4, 4, 0, 0)
    with pytest.raises(hc.HcError):  # 4 x 16 loads in flight exceed the memory counter
        c.set_tuning(0, 0, 4, 8, 4, 2, 4)
    with pytest.raises(hc.HcError):  # epilogue stages only on LDS-staged 4x8 tiles
        c.set_tuning(0, 0, 4, 8, 4, 2, 2, 0, 0, 5)
    with pytest.raises(hc.HcError):  # a depth alone is not a tile
        c.set_tuning(0, 0, 0, 0, 0, 0, 4)
    with pytest.raises(hc.HcError):  # nor is the LDS flag
        c.set_tuning(0, 0, 0, 0, 0, 0, 0, 1)
    if 5 in elogs:
        with pytest.raises(hc.HcError):  # two polynomials per workgroup need inv_elog <= 4
            c.set_tuning(0, 5, 0, 0, 0, 0, 0, 0, 2)


def test_mac_ring_over_many_input_ciphertexts(hc):
    """37 input ciphertexts per output (one channel per ciphertext at N = 1024):
    more than two accumulator folds and a ring turn cut short by the end, for
    every MAC tile and ring depth, against the oracle."""
    N, L, t, B = 1024, 2, 2 ** 17, 5
    c = _ctx(hc, N, L, t)
    spec = W.ConvSpec(37, 9, 28, 28, 3, 1)
    P = layout.plan(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
    assert P.G == 37 and not P.tiled
    g = W.rng(37)
    f = W.gen_filters(g, spec)
    x = W.gen_ct_limbs(g, (B, P.G, 2), c.primes, N)
    r = W.gen_mask(g, (B, spec.c_o, P.ho, P.wo), t)
    ly = hc.Layer(c, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride, f)
    exp = [conv.mask_extract(calg1.alg1_layer(x[b], f, P, c.primes), r[b], P, c.primes, t) for b in range(B)]
    dx, dr = dev(x), dev(r)
    ws = zeros((ly.workspace_words(B, True),))
    for v in MAC_VARIANTS:
        if v[6]:
            continue  # epilogue stages need N >= 4096 (own test below)
        print(f"mac {v}", flush=True)
        c.set_tuning(*mac_tuning(v))
        c0, c1 = zeros(ly.c0_shape(B)), zeros(ly.c1_shape(B))
        ly.conv_masked(dx, dr, c0, c1, B, ws)
        c0, c1 = host(c0), host(c1)
        for b in range(B):
            assert (c0[b] == exp[b][0]).all() and (c1[b] == exp[b][1]).all(), (v, b)


@pytest.mark.parametrize("spec", [W.ConvSpec(148, 13, 28, 28, 3, 1, "g37"), W.ConvSpec(3, 13, 70, 70, 3, 1, "tiled")])
def test_mac_epilogue_stages_match_oracle(hc, spec):
    """MAC variants that apply the inverse NTT's first stages before storing,
    with every inverse shape that starts after them: 37 input ciphertexts per
    output (several folds), a row-tiled layer, c_out = 13 and B = 5 (channels
    and images absent from a workgroup tile), against the oracle."""
    N, L, t, B = 4096, 2, 2 ** 17, 5
    c = _ctx(hc, N, L, t)
    P = layout.plan(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
    assert (P.G == 37) if spec.name == "g37" else P.tiled
    g = W.rng(41)
    f = W.gen_filters(g, spec)
    x = W.gen_ct_limbs(g, (B, P.G, 2), c.primes, N)
    r = W.gen_mask(g, (B, spec.c_o, P.ho, P.wo), t)
    ly = hc.Layer(c, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride, f)
    exp = [conv.mask_extract(calg1.alg1_layer(x[b], f, P, c.primes), r[b], P, c.primes, t) for b in range(B)]
    dx, dr = dev(x), dev(r)
    ws = zeros((ly.workspace_words(B, True),))
    for v in [v for v in MAC_VARIANTS if v[6]]:
        for ie, npw in ((3, 1), (4, 1), (5, 1), (3, 2), (4, 2)):
            print(f"{spec.name} mac {v} inverse e={ie} x{npw}", flush=True)
            c.set_tuning(*mac_tuning(v, ie, npw))
            c0, c1 = zeros(ly.c0_shape(B)), zeros(ly.c1_shape(B))
            ly.conv_masked(dx, dr, c0, c1, B, ws)
            c0, c1 = host(c0), host(c1)
            for b in range(B):
                assert (c0[b] == exp[b][0]).all() and (c1[b] == exp[b][1]).all(), (v, ie, npw, b)


PRUNED = [  # (c_i, c_o, h, w, f, stride): top inverse stages of c0 the layer lets the kernel prune at N = 8192
    W.ConvSpec(40, 9, 7, 7, 3, 1, "7x7"),     # largest extracted index 60: 7 stages
    W.ConvSpec(20, 7, 4, 4, 3, 1, "4x4"),     # index 21: 8 allowed, 7 instantiated
    W.ConvSpec(16, 5, 8, 8, 3, 2, "8x8s2"),   # index 66: 6 allowed, 5 instantiated
]


@pytest.mark.parametrize("spec", PRUNED, ids=lambda s: s.name)
def test_pruned_inverse_shapes_every_output(hc, spec):
    """Small-map layers at N = 8192 whose extracted coefficients let the masked
    inverse NTT prune its top 5 or 7 stages, in every inverse shape the
    autotuner can pick (2^3, 2^4, 2^5 coefficients per thread; one or two
    polynomials per workgroup; with and without the MAC's epilogue stages),
    B = 3 (the last two-polynomial workgroup half empty): every output against
    the oracle."""
    N, L, t, B = 8192, 3, 2 ** 20, 3
    c = _ctx(hc, N, L, t)
    P = layout.plan(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
    g = W.rng(77)
    f = W.gen_filters(g, spec)
    x = W.gen_ct_limbs(g, (B, P.G, 2), c.primes, N)
    r = W.gen_mask(g, (B, spec.c_o, P.ho, P.wo), t)
    ly = hc.Layer(c, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride, f)
    exp = [conv.mask_extract(calg1.alg1_layer(x[b], f, P, c.primes), r[b], P, c.primes, t) for b in range(B)]
    dx, dr = dev(x), dev(r)
    ws = zeros((ly.workspace_words(B, True),))
    cases = [(0, ie, 0, 0, 0, 0, 0, 0, npw) for ie in (3, 4, 5) for npw in (1, 2) if ie <= 4 or npw == 1]
    cases += [mac_tuning(v, ie, npw) for v in MAC_VARIANTS if v[6] for ie, npw in ((3, 2), (4, 2), (4, 1))]
    for tune in cases:
        print(f"{spec.name} tuning {tune}", flush=True)
        c.set_tuning(*tune)
        c0, c1 = zeros(ly.c0_shape(B)), zeros(ly.c1_shape(B))
        ly.conv_masked(dx, dr, c0, c1, B, ws)
        c0, c1 = host(c0), host(c1)
        for b in range(B):
            assert (c0[b] == exp[b][0]).all() and (c1[b] == exp[b][1]).all(), (tune, b)


C0_IN_MAC = [  # (N, L, t, spec): every extracted c0 coefficient below 64, one row tile
    (8192, 3, 2 ** 20, W.ConvSpec(20, 20, 7, 7, 1, 1, "1x1 7x7 G1")),
    (8192, 3, 2 ** 20, W.ConvSpec(400, 37, 7, 7, 1, 1, "1x1 7x7 G3")),
    (8192, 2, 2 ** 17, W.ConvSpec(1800, 20, 7, 7, 3, 1, "3x3 7x7 G18")),
    (8192, 3, 2 ** 20, W.ConvSpec(60, 9, 6, 6, 3, 2, "3x3 6x6 s2")),
    (8192, 3, 2 ** 20, W.ConvSpec(30, 17, 8, 8, 1, 1, "1x1 8x8")),
    (4096, 2, 2 ** 17, W.ConvSpec(90, 20, 4, 4, 5, 1, "5x5 4x4")),
    (16384, 4, 2 ** 24, W.ConvSpec(700, 24, 7, 7, 1, 1, "N16384")),
    (2048, 2, 2 ** 17, W.ConvSpec(40, 12, 5, 5, 3, 1, "N2048")),
    (1024, 1, 3, W.ConvSpec(30, 10, 4, 4, 3, 1, "N1024 L1")),
]


@pytest.mark.parametrize("N,L,t,spec", C0_IN_MAC, ids=lambda v: v.name if hasattr(v, "name") else str(v))
@pytest.mark.parametrize("B", [1, 5])
def test_c0_transform_in_mac_every_output(hc, N, L, t, spec, B):
    """The MAC tiles that carry out c0's masked inverse transform (the six
    stages of each 64-coefficient block, the sum over blocks in splits) and
    leave c1 to a c1-only inverse NTT, on layers whose extracted c0
    coefficients all lie below 64: 1 to 18 input ciphertexts (a fold), ragged channel
    and image tiles, stride 2, N = 1024 to 16384 and 1 to 4 primes, each
    inverse shape for c1: every output against the oracle."""
    c = _ctx(hc, N, L, t)
    P = layout.plan(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
    assert not P.tiled
    e_max = max(P.out_pos(oy, ox)[1] for oy in range(P.ho) for ox in range(P.wo))
    assert e_max < 64, e_max
    g = W.rng(N + spec.c_i + B)
    f = W.gen_filters(g, spec)
    x = W.gen_ct_limbs(g, (B, P.G, 2), c.primes, N)
    r = W.gen_mask(g, (B, spec.c_o, P.ho, P.wo), t)
    ly = hc.Layer(c, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride, f)
    exp = [conv.mask_extract(calg1.alg1_layer(x[b], f, P, c.primes), r[b], P, c.primes, t) for b in range(B)]
    dx, dr = dev(x), dev(r)
    ws = zeros((ly.workspace_words(B, True),))
    elogs = (4, 5) if N == 16384 else (3, 4)  # shapes every ring size has
    for v in [v for v in MAC_VARIANTS if v[6] == 6]:
        for ie, npw in [(e, 1) for e in elogs] + [(4, 2)]:
            print(f"{spec.name} B={B} mac {v} c1 inverse e={ie} x{npw}", flush=True)
            c.set_tuning(*mac_tuning(v, ie, npw))
            c0, c1 = zeros(ly.c0_shape(B)), zeros(ly.c1_shape(B))
            ly.conv_masked(dx, dr, c0, c1, B, ws)
            c0, c1 = host(c0), host(c1)
            for b in range(B):
                assert (c0[b] == exp[b][0]).all(), (v, ie, npw, b, "c0")
                assert (c1[b] == exp[b][1]).all(), (v, ie, npw, b, "c1")


def test_resnet18_cifar_every_output(hc):
    """ResNet-18/CIFAR at N = 8192, 3 primes, t = 2^20, one image, one launch
    sequence per layer with launch shapes autotuned at B = 1 (as the benchmark's
    plain leg): every output coefficient of every layer (c0_ext and c1_out)
    against the oracle (Algorithm 1 in C, then mask and extraction)."""
    import torch
    N, L, t, B = 8192, 3, 2 ** 20, 1
    c = _ctx(hc, N, L, t)
    specs = W.resnet18_cifar()
    g = W.rng(1818)
    filters = [W.gen_filters(g, s) for s in specs]
    layers = [hc.Layer(c, s.c_i, s.c_o, s.h, s.w, s.f_w, s.stride, f) for s, f in zip(specs, filters)]
    plans = [layout.plan(N, s.c_i, s.c_o, s.h, s.w, s.f_w, s.stride) for s in specs]
    xs = [W.gen_ct_limbs(g, (B, P.G, 2), c.primes, N) for P in plans]
    rs = [W.gen_mask(g, (B, s.c_o, P.ho, P.wo), t) for s, P in zip(specs, plans)]
    dx, dr = [dev(x) for x in xs], [dev(r) for r in rs]
    c0 = [zeros(ly.c0_shape(B)) for ly in layers]
    c1 = [zeros(ly.c1_shape(B)) for ly in layers]
    bt = hc.Batch(c, layers, B)
    print("autotune at B=1", flush=True)
    bt.autotune(dx, dr, c0, c1)
    bt.close()
    ws = zeros((max(ly.workspace_words(B, True) for ly in layers),))
    for k, (s, ly, P) in enumerate(zip(specs, layers, plans)):
        assert ly.tuning()[0] == B
        c0[k].zero_()
        c1[k].zero_()
        ly.conv_masked(dx[k], dr[k], c0[k], c1[k], B, ws)
    torch.cuda.synchronize()
    for k, (s, f, P) in enumerate(zip(specs, filters, plans)):
        print(f"r18-cifar layer {k} {s.name}: every output", flush=True)
        y = calg1.alg1_layer(xs[k][0], f, P, c.primes)
        e0, e1 = conv.mask_extract(y, rs[k][0], P, c.primes, t)
        assert (host(c0[k])[0] == e0).all(), f"layer {k}: c0_ext differs"
        assert (host(c1[k])[0] == e1).all(), f"layer {k}: c1_out differs"
    for ly in layers:
        ly.close()
