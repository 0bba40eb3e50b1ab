"""Input validation of the interface: inputs must be canonical residues.
hc_check_residues counts the words that are not; with HC_CHECK_INPUTS=1 set
when a context is created, the conv calls refuse such inputs with HC_EINVAL
and otherwise give the same bits as an unchecked context."""
import os

import numpy as np
import pytest

from oracle import conv, calg1, layout
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


def test_check_residues_counts_noncanonical_words(hc):
    N, L = 4096, 3
    c = hc.Context(N, L, 2 ** 17)
    g = W.rng(11)
    x = W.gen_ct_limbs(g, (5, 2), c.primes, N)  # [5][2][L][N]
    assert c.check_residues(dev(x)) == 0
    x[0, 0, 1, 7] = c.primes[1]          # equal to its prime: not canonical
    x[4, 1, 2, N - 1] = 0xFFFFFFFF       # far out of range
    x[2, 0, 0, 3] = c.primes[0] - 1      # the largest canonical value
    assert c.check_residues(dev(x)) == 2
    # a value below another limb's prime but not its own
    x2 = W.gen_ct_limbs(g, (1, 1), c.primes, N)
    lo, hi = min(c.primes), max(c.primes)
    l_lo = c.primes.index(lo)
    x2[0, 0, l_lo, 0] = hi - 1 if hi - 1 >= lo else lo
    assert c.check_residues(dev(x2)) == 1
    with pytest.raises(ValueError):
        c.check_residues(zeros((N * L + 1,)))


def test_conv_refuses_noncanonical_inputs_when_checking(hc, monkeypatch):
    N, L, t, B = 1024, 2, 2 ** 17, 2
    spec = W.ConvSpec(5, 3, 14, 14, 3, 1)
    P = layout.plan(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
    g = W.rng(12)
    f = W.gen_filters(g, spec)
    monkeypatch.setenv("HC_CHECK_INPUTS", "1")
    c = hc.Context(N, L, t)
    monkeypatch.delenv("HC_CHECK_INPUTS")
    x = W.gen_ct_limbs(g, (B, P.G, 2), c.primes, N)
    r = W.gen_mask(g, (B, spec.c_o, P.ho, P.wo), t)
    ly = hc.Layer(c, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride, f)
    ws = zeros((ly.workspace_words(B, True),))
    c0, c1 = zeros(ly.c0_shape(B)), zeros(ly.c1_shape(B))
    ly.conv_masked(dev(x), dev(r), c0, c1, B, ws)  # canonical: accepted, oracle bits
    c0, c1 = host(c0), host(c1)
    for b in range(B):
        e0, e1 = conv.mask_extract(calg1.alg1_layer(x[b], f, P, c.primes), r[b], P, c.primes, t)
        assert (c0[b] == e0).all() and (c1[b] == e1).all(), b
    bad = x.copy()
    bad[1, P.G - 1, 1, 0, N - 1] = c.primes[0]
    with pytest.raises(hc.HcError) as err:
        ly.conv_masked(dev(bad), dev(r), zeros(ly.c0_shape(B)), zeros(ly.c1_shape(B)), B, ws)
    assert err.value.status == -1  # HC_EINVAL
    with pytest.raises(hc.HcError):
        ly.conv(dev(bad), zeros(ly.out_shape(B)), B, zeros((ly.workspace_words(B, False),)))
