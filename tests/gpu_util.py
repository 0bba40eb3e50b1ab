"""Helpers shared by the GPU tests: host <-> device copies of uint32 residues,
and sampled comparison of a layer's outputs against the oracle."""
import numpy as np

from oracle import calg1, conv


def dev(a):
    import torch
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32)).cuda()


def host(t):
    return t.cpu().numpy().view(np.uint32)


def zeros(shape):
    import torch
    return torch.zeros(tuple(shape), dtype=torch.int32, device="cuda")


def check_layer_points(P, primes, t, x_img, f, mask_img, c0_img, c1_img, g, npts=64):
    """Compare npts sampled c1 coefficients and npts sampled extracted c0
    outputs of one image against Algorithm 1's closed form (oracle)."""
    L = len(primes)
    # c1: any coefficient of any output ciphertext
    i = g.integers(0, P.c_o, size=npts)
    tau = g.integers(0, P.T, size=npts)
    l = g.integers(0, L, size=npts)
    m = g.integers(0, P.n, size=npts)
    exp = calg1.alg1_points(x_img, f, P, primes, i, tau, np.ones(npts, dtype=np.int64), l, m)
    got = c1_img[i * P.T + tau, l, m]
    assert (got == exp).all(), f"c1 mismatch at {np.nonzero(got != exp)[0][:5]}"
    # c0: extracted output pixels with the mask added
    i = g.integers(0, P.c_o, size=npts)
    oy = g.integers(0, P.ho, size=npts)
    ox = g.integers(0, P.wo, size=npts)
    l = g.integers(0, L, size=npts)
    pos = [P.out_pos(int(a), int(b)) for a, b in zip(oy, ox)]
    taus = np.array([p[0] for p in pos])
    es = np.array([p[1] for p in pos])
    y = calg1.alg1_points(x_img, f, P, primes, i, taus, np.zeros(npts, dtype=np.int64), l, es)
    exp = np.array([conv.mask_add(int(y[k]), int(mask_img[i[k], oy[k], ox[k]]), int(l[k]), primes, t)
                    for k in range(npts)], dtype=np.uint32)
    got = c0_img[i, l, oy, ox]
    assert (got == exp).all(), f"c0 mismatch at {np.nonzero(got != exp)[0][:5]}"
