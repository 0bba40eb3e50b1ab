"""hc_conv_masked_noalloc (the masked convolution without a workspace, for
callers that cannot allocate): through the C ABI, its outputs equal
hc_conv_masked's bit for bit on two calls in a row, the second with a smaller
input, and a layer whose scratch exceeds the fixed array is refused before any
device work."""
import numpy as np
import pytest

from oracle import calg1, conv, layout
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


def _case(hc, c, spec, B, seed):
    P = layout.plan(c.N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
    g = W.rng(seed)
    f = W.gen_filters(g, spec)
    x = W.gen_ct_limbs(g, (B, P.G, 2), c.primes, c.N)
    r = W.gen_mask(g, (B, spec.c_o, P.ho, P.wo), c.t)
    ly = hc.Layer(c, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride, f)
    return P, f, x, r, ly


def _both(ly, x, r, B):
    """(noalloc outputs, workspace outputs) on the same inputs."""
    import torch
    dx, dr = dev(x), dev(r)
    a0, a1 = zeros(ly.c0_shape(B)), zeros(ly.c1_shape(B))
    ly.conv_masked_noalloc(dx, dr, a0, a1, B)
    b0, b1 = zeros(ly.c0_shape(B)), zeros(ly.c1_shape(B))
    ly.conv_masked(dx, dr, b0, b1, B, zeros((ly.workspace_words(B, True),)))
    torch.cuda.synchronize()
    return (host(a0), host(a1)), (host(b0), host(b1))


def test_noalloc_matches_workspace_path_on_two_calls(hc):
    """A ResNet-18/CIFAR-shaped layer at N = 8192 on 3 images (most of the
    scratch array), then a smaller layer on one image: each call's outputs equal
    hc_conv_masked's, and the first also the oracle's."""
    N, L, t = 8192, 3, 2 ** 20
    c = hc.Context(N, L, t)
    spec1 = W.ConvSpec(64, 128, 32, 32, 3, 2, "big")
    P1, f1, x1, r1, ly1 = _case(hc, c, spec1, 3, 901)
    assert ly1.workspace_words(3, True) * 4 <= hc.Layer.NOALLOC_SCRATCH_BYTES
    print("noalloc call 1: 64->128 32x32 s2, B=3", flush=True)
    (a0, a1), (b0, b1) = _both(ly1, x1, r1, 3)
    assert (a0 == b0).all() and (a1 == b1).all()
    e0, e1 = conv.mask_extract(calg1.alg1_layer(x1[2], f1, P1, c.primes), r1[2], P1, c.primes, t)
    assert (a0[2] == e0).all() and (a1[2] == e1).all()
    spec2 = W.ConvSpec(16, 8, 16, 16, 3, 1, "small")
    P2, f2, x2, r2, ly2 = _case(hc, c, spec2, 1, 902)
    print("noalloc call 2: 16->8 16x16, B=1", flush=True)
    (a0, a1), (b0, b1) = _both(ly2, x2, r2, 1)
    assert (a0 == b0).all() and (a1 == b1).all()
    e0, e1 = conv.mask_extract(calg1.alg1_layer(x2[0], f2, P2, c.primes), r2[0], P2, c.primes, t)
    assert (a0[0] == e0).all() and (a1[0] == e1).all()
    ly1.close()
    ly2.close()
    c.close()


def test_noalloc_refuses_a_layer_beyond_its_scratch(hc):
    """ResNet-50's last 1x1 layer (2048 output ciphertexts) needs 403 MB of
    scratch for one image: refused with HC_EINVAL, nothing launched."""
    N, L, t = 8192, 3, 2 ** 20
    c = hc.Context(N, L, t)
    spec = W.ConvSpec(512, 2048, 7, 7, 1, 1, "s4.c3")
    P = layout.plan(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
    ly = hc.Layer(c, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride,
                  np.zeros((spec.c_o, spec.c_i, 1, 1), dtype=np.int8))
    assert ly.workspace_words(1, True) * 4 > hc.Layer.NOALLOC_SCRATCH_BYTES
    c0, c1 = zeros(ly.c0_shape(1)), zeros(ly.c1_shape(1))
    with pytest.raises(hc.HcError) as e:
        ly.conv_masked_noalloc(zeros(ly.in_shape(1)), zeros(ly.mask_shape(1)), c0, c1, 1)
    assert e.value.status == -1 and "scratch" in str(e.value)
    assert P.O == 2048
    ly.close()
    c.close()


def test_noalloc_with_c0_transform_in_the_mac(hc):
    """A 7x7 layer whose MAC carries out c0's transform (mac_pre = 6: c0's
    partial sums in the scratch's Yhat, c1-only inverse NTT, finishing pass):
    two no-allocation calls in a row (3 images, then 1) equal the workspace
    path's and the oracle's outputs."""
    N, L, t = 8192, 3, 2 ** 20
    c = hc.Context(N, L, t)
    c.set_tuning(0, 0, 4, 8, 2, 2, 4, 2, 0, 6)
    spec = W.ConvSpec(400, 40, 7, 7, 1, 1, "7x7")
    for B, seed in ((3, 903), (1, 904)):
        P, f, x, r, ly = _case(hc, c, spec, B, seed)
        assert ly.workspace_words(B, True) * 4 <= hc.Layer.NOALLOC_SCRATCH_BYTES
        print(f"noalloc with c0 in the MAC: 400->40 7x7, B={B}", flush=True)
        (a0, a1), (b0, b1) = _both(ly, x, r, B)
        assert (a0 == b0).all() and (a1 == b1).all()
        e0, e1 = conv.mask_extract(calg1.alg1_layer(x[B - 1], f, P, c.primes), r[B - 1], P, c.primes, t)
        assert (a0[B - 1] == e0).all() and (a1[B - 1] == e1).all()
        ly.close()
    c.close()
