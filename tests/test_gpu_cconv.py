"""The conventional convolution on the GPU (batch encoding, HRot with key
switching, PMult) against the oracle (oracle/hrot.py): rotation-order slot
encoding both ways, every output coefficient of the packed convolution for
switching keys generated on the GPU from the oracle's random inputs, and at
N = 8192 (a Table 9 layer shape) the decrypt invariant: decrypting and
decoding the output gives the plain convolution mod t."""
import numpy as np
import pytest

from oracle import bfv, conv, hrot, params
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


def test_rotation_order_encoding_matches_oracle(hc):
    N, L, t = 1024, 3, 12289
    c = hc.Context(N, L, t)
    g = W.rng(11)
    z = g.integers(0, t, size=(3, 2, N // 2))
    p = zeros((3, N))
    c.rot_encode(dev(z.reshape(3, N)), p)
    ph = host(p)
    for k in range(3):
        assert (ph[k] == hrot.rot_encode(z[k], t, N)).all(), k
    zz = zeros((3, N))
    c.rot_decode(p, zz, zeros((3 * N,)))
    assert (host(zz).reshape(3, 2, N // 2) == z).all()
    c.close()


CCASES = [  # (N, c_in, c_out, h, w, f, decomposition bits)
    (1024, 5, 6, 16, 16, 3, 10),   # c_r = 2 (blocks of 256), two input and output ciphertexts
    (1024, 7, 3, 8, 8, 1, 10),     # 1x1, c_r = 8, one ciphertext each
    (1024, 3, 2, 16, 32, 3, 6),    # one channel per slot row (h w = N/2), 6-bit digits
]


@pytest.mark.parametrize("case", CCASES)
def test_conventional_conv_matches_oracle(hc, case):
    N, ci, co, h, w, f, T = case
    L, t = 3, 12289
    c = hc.Context(N, L, t)
    primes = c.primes
    CL = hrot.CLayout(N, ci, co, h, w, f)
    g = W.rng(sum(case))
    s = bfv.sample_secret(g, N)
    filt = g.integers(-128, 128, size=(co, ci, f, f)).astype(np.int8)
    cc = hc.CConv(c, ci, co, h, w, f, filt, T)
    lay = cc.layout
    assert (lay.c_r, lay.block, lay.c_n, lay.g_in, lay.g_out) == (CL.c_r, CL.bsz, CL.c_n, CL.G_in, CL.G_out)
    assert cc.galois == [r[5] for r in CL.rotations]
    R, LD = lay.rotations, lay.digits
    a = W.gen_ct_limbs(g, (R * LD,), primes, N).reshape(R, LD, L, N)
    e = np.stack([np.stack([bfv.sample_error(g, N) for _ in range(LD)]) for _ in range(R)]).astype(np.int32)
    keys_o = {ri: hrot.switching_key(s, gal, a[ri], e[ri], primes, T) for ri, gal in enumerate(cc.galois)
              if gal != 1}
    a_in = g.integers(0, t, size=(ci, h, w))
    zin = CL.encode_input(a_in, t)
    cts = []
    for k in range(CL.G_in):
        mc = np.array([params.centred(int(v), t) for v in hrot.rot_encode(zin[k], t, N)])
        cts.append(bfv.encrypt_sk(mc, s, bfv.sample_a(g, primes, N), bfv.sample_error(g, N), primes, t))
    cts = np.stack(cts)
    print(f"oracle {case}", flush=True)
    want = hrot.conventional_conv(cts, filt, CL, keys_o, primes, t, T)
    import torch
    sk = dev(np.stack([np.asarray(s) % q for q in primes]))
    keys = zeros((cc.keys_words(),))
    cc.keygen(sk, dev(a), torch.from_numpy(e).cuda(), keys, zeros((cc.keygen_workspace_words(),)))
    out = zeros((1, CL.G_out, 2, L, N))
    print(f"gpu {case}", flush=True)
    cc.run(keys, dev(cts[None]), out, 1, zeros((cc.workspace_words(1),)))
    got = host(out)[0]
    assert (got == want).all(), np.argwhere(got != want)[:5]
    # and the decrypt invariant
    zout = np.stack([hrot.rot_decode(np.array(bfv.decrypt(got[o], s, primes, t)), t, N) for o in range(CL.G_out)])
    assert (CL.decode_output(zout) == conv.plain_conv_mod_t(a_in, filt, 1, t)).all()
    cc.close()
    c.close()


def test_conventional_conv_decrypt_invariant_full_size(hc):
    """(16x16, 64 -> 64, 3x3) at N = 8192, 3 primes, t = 786433, 10-bit digits:
    keys, encryption, the convolution, decryption and decoding on the GPU;
    the decoded output equals the plain convolution mod t at every pixel."""
    import torch
    N, L, t, T = 8192, 3, 786433, 10
    ci, co, h, w, f = 64, 64, 16, 16, 3
    c = hc.Context(N, L, t)
    primes = c.primes
    CL = hrot.CLayout(N, ci, co, h, w, f)
    g = W.rng(916)
    filt = g.integers(-128, 128, size=(co, ci, f, f)).astype(np.int8)
    cc = hc.CConv(c, ci, co, h, w, f, filt, T)
    R, LD = cc.layout.rotations, cc.layout.digits
    tg = torch.Generator(device="cuda")
    tg.manual_seed(916)
    s = torch.randint(-1, 2, (N,), generator=tg, device="cuda", dtype=torch.int64)
    sk = torch.stack([torch.remainder(s, q) for q in primes]).to(torch.int32).contiguous()
    a = W.gen_ct_limbs_torch(tg, (R * LD,), primes, N, "cuda")
    e = torch.randint(-8, 9, (R * LD, N), generator=tg, device="cuda", dtype=torch.int32)
    keys = zeros((cc.keys_words(),))
    print("keygen", flush=True)
    cc.keygen(sk, a, e, keys, zeros((cc.keygen_workspace_words(),)))
    a_in = g.integers(0, t, size=(ci, h, w))
    zin = CL.encode_input(a_in, t).reshape(CL.G_in, N)
    p = zeros((CL.G_in, N))
    c.rot_encode(dev(zin), p)
    az = W.gen_ct_limbs_torch(tg, (CL.G_in,), primes, N, "cuda")
    ez = torch.randint(-8, 9, (CL.G_in, N), generator=tg, device="cuda", dtype=torch.int32)
    ct0 = zeros((CL.G_in, 2, L, N))
    c.encrypt_zero(az, sk, ez, ct0, zeros(((CL.G_in + 1) * L * N,)))
    ct = zeros((1, CL.G_in, 2, L, N))
    c.encrypt_plain(p, ct0, ct[0])
    out = zeros((1, CL.G_out, 2, L, N))
    print("conventional conv", flush=True)
    cc.run(keys, ct, out, 1, zeros((cc.workspace_words(1),)))
    m = zeros((CL.G_out, N))
    c.decrypt(out[0], sk, m, zeros(((CL.G_out + 1) * L * N,)))
    zo = zeros((CL.G_out, N))
    c.rot_decode(m, zo, zeros((CL.G_out * N,)))
    got = CL.decode_output(host(zo).reshape(CL.G_out, 2, N // 2))
    assert (got == conv.plain_conv_mod_t(a_in, filt, 1, t)).all()
    cc.close()
    c.close()
