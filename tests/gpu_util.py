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


def freivalds_check(P, primes, delta_mod_q, t, x_img, f, mask_img, c0_img, c1_img, g):
    """Every output of one image against the oracle at once: for random rho
    (one residue per output channel and limb), sum_i rho_i c1_(i,tau) must equal
    the oracle's combination of Algorithm 1's c1 outputs at every coefficient,
    and sum_i rho_i (c0_ext_i - Delta_l r_i) must equal its c0 combination at
    every extracted coefficient (tolerance 0). A wrong value anywhere passes
    with probability at most 1/q_l per compared coefficient.

    x_img: host input ciphertexts [G][2][L][n]; mask_img, c0_img, c1_img: the
    image's device tensors (int32 views of uint32). The combination on the
    device side is test arithmetic in int64 torch ops; rhs comes from
    oracle.calg1.freivalds_rhs."""
    import torch
    L = len(primes)
    rho = [g.integers(0, q, size=P.c_o) for q in primes]
    rhs = calg1.freivalds_rhs(x_img, f, rho, P, primes)  # [T][2][L][n]
    dev = c1_img.device
    u32 = lambda v: v.to(torch.int64) & 0xFFFFFFFF
    c1 = u32(c1_img).view(P.c_o, P.T, L, P.n)
    c0 = u32(c0_img).view(P.c_o, L, P.ho, P.wo)
    r = u32(mask_img).view(P.c_o, P.ho, P.wo)
    rc = torch.where(r > t // 2, r - t, r)  # centred lift of the mask
    taus = np.zeros((P.ho, P.wo), dtype=np.int64)
    es = np.zeros((P.ho, P.wo), dtype=np.int64)
    for oy in range(P.ho):
        for ox in range(P.wo):
            taus[oy, ox], es[oy, ox] = P.out_pos(oy, ox)
    for l, q in enumerate(primes):
        rl = torch.tensor(rho[l], dtype=torch.int64, device=dev)
        lhs1 = ((c1[:, :, l, :] * rl[:, None, None]) % q).sum(0) % q  # [T][n]
        exp1 = rhs[:, 1, l, :].astype(np.int64)
        got1 = lhs1.cpu().numpy()
        assert (got1 == exp1).all(), f"c1 combination differs at limb {l}: {np.argwhere(got1 != exp1)[:4]}"
        y0 = (c0[:, l] - (delta_mod_q[l] * (rc % q)) % q) % q  # c0 before the mask, [c_o][ho][wo]
        lhs0 = ((y0 * rl[:, None, None]) % q).sum(0) % q
        exp0 = rhs[taus, 0, l, es].astype(np.int64)
        got0 = lhs0.cpu().numpy()
        assert (got0 == exp0).all(), f"c0 combination differs at limb {l}: {np.argwhere(got0 != exp0)[:4]}"
