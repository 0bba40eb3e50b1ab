"""Serving benchmark: Poisson arrivals of private-inference requests.

    python -m paper_2401_16732_amd.serve [--duration S] [--mix 0.5] ...

Two networks are resident on one GPU at N = 8192 with 3 primes (t = 2^20):
ResNet-18 on 32x32 inputs and ResNet-50 on 224x224 inputs, with their NTT-domain
weights and twiddles encoded once. A request is one image through every
convolution layer of its network (the HE part of one private inference);
`mix` is the fraction of ResNet-50 requests. The server (hc_server_*) admits
requests by HBM arena space and batches the next layer of all in-flight
requests of the same network and layer together.

First the saturation throughput is measured (a burst of requests submitted at
once); then arrivals are Poisson at rates swept from 0.1x to 1.2x that
throughput. For every rate one JSON line reports throughput and the p50 / p99
of request latency (submission to completion seen by the host loop).
Inputs are synthetic (uniform residues and masks); each request reads one of
a few resident input sets of its network (the client's upload).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--duration", type=float, default=8.0, help="seconds of arrivals per rate")
    ap.add_argument("--mix", type=float, default=0.5, help="fraction of ResNet-50 requests")
    ap.add_argument("--rates", default="0.1,0.3,0.5,0.7,0.9,1.0,1.2", help="fractions of saturation throughput")
    ap.add_argument("--arena-gib", type=float, default=160.0)
    ap.add_argument("--max-batch", type=int, default=16)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--max-inflight", type=int, default=8, help="launch groups on the GPU at once (0: no limit)")
    ap.add_argument("--burst", type=int, default=64, help="requests in the saturation burst")
    ap.add_argument("--sets", type=int, default=2, help="distinct input sets per network")
    ap.add_argument("--seed", type=int, default=4)
    return ap.parse_args()


def build_nets(hconv, W, ctx, g, names=("resnet18_cifar", "resnet50_224"), nets=None):
    """Resident layers (NTT-domain weights) of each named network; entries
    already in `nets` are kept."""
    nets = dict(nets or {})
    for name in names:
        if name not in nets:
            specs = W.NETS[name]()
            nets[name] = [hconv.Layer(ctx, s.c_i, s.c_o, s.h, s.w, s.f_w, s.stride, W.gen_filters(g, s))
                          for s in specs]
    return nets


def request_work(nets, N, L):
    """Algorithmic work of one request of each network (one image through
    every layer): NTT butterflies (forward of the inputs, inverse of the
    outputs) and multiply-accumulate terms."""
    import math
    logn = int(math.log2(N))
    out = {}
    for name, layers in nets.items():
        bfly = mac = 0
        for ly in layers:
            lay = ly.layout
            bfly += (lay.in_cts + lay.out_cts) * 2 * L * (N // 2) * logn
            mac += lay.out_cts * lay.w_cts * 2 * L * N
        out[name] = {"butterflies": bfly, "mac": mac}
    return out


def sweep(hconv, W, ctx, nets, *, mix=0.5, rates=(0.1, 0.3, 0.5, 0.7, 0.9, 1.0, 1.2), duration=8.0,
          arena_gib=160.0, max_batch=16, streams=4, max_inflight=8, burst=64, sets=2, seed=4,
          bfly_peak=None, mac_peak=None, log=None):
    """Saturation burst, then Poisson arrivals at each rate fraction of it.
    Returns {"setup", "saturation", "rates": [...]}; with the VALU peaks given,
    each rate also reports the served work's ideal VALU time over the wall
    time (served_alu_frac)."""
    import torch
    dev = torch.device("cuda", ctx.device)
    N, L, t = ctx.N, ctx.L, ctx.t
    srv = hconv.Server(ctx, int(arena_gib * 2 ** 30), max_batch, streams, max_inflight)
    nid = {name: srv.add_net(layers) for name, layers in nets.items()}
    tg = torch.Generator(device=dev)
    tg.manual_seed(seed)
    inputs = {}
    for name, layers in nets.items():
        inputs[name] = []
        for _ in range(sets):
            x = [W.gen_ct_limbs_torch(tg, ly.in_shape(1)[1:3], ctx.primes, N, dev) for ly in layers]
            m = [torch.randint(0, t, ly.mask_shape(1)[1:], generator=tg, device=dev, dtype=torch.int32)
                 for ly in layers]
            inputs[name].append((x, m))
    torch.cuda.synchronize()
    work = request_work(nets, N, L)
    setup = {"networks": {k: {"layers": len(v), "request_bytes": srv.request_bytes(nid[k]), **work[k]}
                          for k, v in nets.items()},
             "arena_gib": arena_gib, "max_batch": max_batch, "streams": streams, "max_inflight": max_inflight,
             "mix_resnet50": mix}
    rng = np.random.default_rng(seed)
    names = sorted(nets)

    def pick():
        name = "resnet50_224" if ("resnet50_224" in nets and rng.random() < mix) else \
            [n for n in names if n != "resnet50_224"][0]
        x, m = inputs[name][int(rng.integers(0, sets))]
        return name, x, m

    def drive(arrivals):
        """arrivals: sorted submission times (s, relative). Returns latencies (s),
        the makespan and the requests' network names."""
        start = time.perf_counter()
        sub, lat = {}, []
        k, n = 0, len(arrivals)
        kinds = [pick() for _ in range(n)]
        while len(lat) < n:
            now = time.perf_counter() - start
            while k < n and arrivals[k] <= now:
                name, x, m = kinds[k]
                rid = srv.submit(nid[name], x, m)
                sub[rid] = (start + arrivals[k], name)
                k += 1
            srv.step()
            for rid in srv.poll():
                t_sub, _ = sub.pop(rid)
                lat.append(time.perf_counter() - t_sub)
                srv.release(rid)
        return np.array(lat), time.perf_counter() - start, [kd[0] for kd in kinds]

    def alu_frac(kinds, span):
        if not bfly_peak or not mac_peak:
            return None
        ideal = sum(work[k]["butterflies"] / bfly_peak + work[k]["mac"] / mac_peak for k in kinds)
        return round(ideal / span, 4)

    # warm-up and saturation: a burst submitted at once
    drive([0.0] * 4)
    lat, span, kinds = drive([0.0] * burst)
    sat = burst / span
    res = {"setup": setup,
           "saturation": {"requests": burst, "seconds": round(span, 3), "requests_per_s": round(sat, 2),
                          "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
                          "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
                          "served_alu_frac": alu_frac(kinds, span)},
           "rates": []}
    if log:
        log({"saturation": res["saturation"]})
    for frac in rates:
        lam = frac * sat
        n = max(8, int(lam * duration))
        arrivals = np.cumsum(rng.exponential(1.0 / lam, size=n)).tolist()
        before = srv.stats()
        lat, span, kinds = drive(arrivals)
        after = srv.stats()
        groups = after["groups"] - before["groups"]
        images = after["images"] - before["images"]
        row = {"rate_fraction": frac, "offered_per_s": round(lam, 2), "requests": n,
               "throughput_per_s": round(n / span, 2),
               "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
               "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
               "mean_group_images": round(images / max(1, groups), 2),
               "served_alu_frac": alu_frac(kinds, span)}
        res["rates"].append(row)
        if log:
            log(row)
    srv.sync()
    srv.close()
    return res


def main():
    a = parse()
    import torch
    from . import hconv, workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    N, L, t = 8192, 3, 2 ** 20
    ctx = hconv.Context(N, L, t)
    g = W.rng(a.seed)
    t0 = time.perf_counter()
    nets = build_nets(hconv, W, ctx, g)
    torch.cuda.synchronize()
    enc_ms = (time.perf_counter() - t0) * 1e3
    print(json.dumps({"weight_encode_ms": round(enc_ms, 1)}), flush=True)
    sweep(hconv, W, ctx, nets, mix=a.mix, rates=[float(v) for v in a.rates.split(",")], duration=a.duration,
          arena_gib=a.arena_gib, max_batch=a.max_batch, streams=a.streams, max_inflight=a.max_inflight,
          burst=a.burst, sets=a.sets, seed=a.seed, log=lambda d: print(json.dumps(d), flush=True))
    return 0


if __name__ == "__main__":
    sys.exit(main())
