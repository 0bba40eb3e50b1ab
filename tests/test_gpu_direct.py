"""Flash's coefficient-domain convolution (Algorithm 1 as written) on the GPU,
through the C ABI: every output bit-exact against the oracle on small layers,
equal to the NTT path at a ResNet-50 layer's full size (with sampled outputs
against the oracle's closed form), and refused on tiled layers."""
import numpy as np
import pytest

from oracle import calg1, conv, layout
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


@pytest.mark.parametrize("N,L,t,shape", [
    (1024, 2, 2 ** 17, (5, 3, 14, 14, 3, 1)),     # one ciphertext, ragged packing
    (1024, 3, 65537, (30, 17, 9, 9, 3, 1)),       # 4 ciphertexts, 17 channels (two channel groups)
    (1024, 2, 2 ** 17, (6, 4, 15, 15, 1, 2)),     # 1x1 stride 2: client subsampling
    (1024, 1, 2 ** 20, (3, 2, 13, 13, 3, 2)),     # 3x3 stride 2
    (4096, 2, 2 ** 17, (16, 16, 16, 16, 3, 1)),
    (2048, 4, 2 ** 17, (2, 3, 20, 20, 5, 1)),     # 5x5
])
def test_direct_conv_matches_oracle(hc, N, L, t, shape):
    c = hc.Context(N, L, t)
    spec = W.ConvSpec(*shape)
    P = layout.plan(N, *shape)
    assert not P.tiled
    g = W.rng(99)
    f = W.gen_filters(g, spec)
    ly = hc.Layer(c, *shape, f)
    B = 2
    x = W.gen_ct_limbs(g, (B, P.G, 2), c.primes, N)
    r = W.gen_mask(g, (B, P.c_o, P.ho, P.wo), t)
    c0, c1 = zeros(ly.c0_shape(B)), zeros(ly.c1_shape(B))
    print(f"direct conv N={N} L={L} {shape}", flush=True)
    ly.conv_masked_direct(dev(x), dev(r), c0, c1, B)
    c0, c1 = host(c0), host(c1)
    for b in range(B):
        e0, e1 = conv.mask_extract(calg1.alg1_layer(x[b], f, P, c.primes), r[b], P, c.primes, t)
        assert (c0[b] == e0).all() and (c1[b] == e1).all(), b


def test_direct_conv_refuses_tiled_layers(hc):
    c = hc.Context(1024, 2, 2 ** 17)
    shape = (2, 2, 40, 40, 3, 1)
    ly = hc.Layer(c, *shape, W.gen_filters(W.rng(1), W.ConvSpec(*shape)))
    with pytest.raises(hc.HcError) as err:
        ly.conv_masked_direct(zeros(ly.in_shape(1)), zeros(ly.mask_shape(1)), zeros(ly.c0_shape(1)),
                              zeros(ly.c1_shape(1)), 1)
    assert err.value.status == -2


def test_direct_conv_equals_ntt_path_resnet50_1x1(hc):
    """ResNet-50 conv2_x 1x1 layer 64 -> 256 at 56 x 56 (c_n = 2), N = 8192,
    L = 3, t = 2^20, one image: both paths give the same bits everywhere, and
    sampled outputs match the oracle's closed form."""
    N, L, t, B = 8192, 3, 2 ** 20, 1
    shape = (64, 256, 56, 56, 1, 1)
    c = hc.Context(N, L, t)
    P = layout.plan(N, *shape)
    g = W.rng(256)
    f = W.gen_filters(g, W.ConvSpec(*shape))
    ly = hc.Layer(c, *shape, f)
    x = W.gen_ct_limbs(g, (B, P.G, 2), c.primes, N)
    r = W.gen_mask(g, (B, P.c_o, P.ho, P.wo), t)
    xd, rd = dev(x), dev(r)
    a0, a1 = zeros(ly.c0_shape(B)), zeros(ly.c1_shape(B))
    ly.conv_masked(xd, rd, a0, a1, B, zeros((ly.workspace_words(B, True),)))
    d0, d1 = zeros(ly.c0_shape(B)), zeros(ly.c1_shape(B))
    print("direct conv ResNet-50 1x1 64->256 56x56", flush=True)
    ly.conv_masked_direct(xd, rd, d0, d1, B)
    a0, a1, d0, d1 = host(a0), host(a1), host(d0), host(d1)
    assert (a0 == d0).all() and (a1 == d1).all()
    check_layer_points(P, c.primes, t, x[0], f, r[0], d0[0], d1[0], W.rng(5))
