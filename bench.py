#!/usr/bin/env python3
"""Benchmark: HE convolution of a whole ResNet-50 (224x224) on one MI355X.

One step = every convolution layer of the network (53 layers) on a batch of B
images, each layer computed as forward NTT -> multiply-accumulate against
resident NTT-domain weights -> inverse NTT with the server mask added and the
output coefficients extracted, replayed as one HIP graph. Inputs (ciphertexts,
masks) are resident in HBM before the timed region. Reported:

  value                ms of HE convolution per ResNet-50 image (batched graph)
  ms_per_step_spread   median, p10 and p90 of the single-step times
  plain_ms_per_image   the same work per image with one launch sequence per
                       layer at B = 1 (stream order, no graph)
  plain_hybrid_ms_per_image  the plain path with Flash's coefficient-domain
                       conv (Algorithm 1 as written) on the layers where it
                       beats the NTT path at one image
  speedup_vs_plain     best plain leg / batched (both legs autotuned for their
                       own batch size)
  modmul_per_s         algorithmic modular multiplies (NTT butterflies + MAC)
                       per second, batched
  valu_probe           register-only VALU rates measured on the device
                       (hc_valu_probe): the lane rates behind the ALU peak
  roofline             the dominant kernel against the VALU / HBM ceiling
  configs              the other workloads, each timed apart: ResNet-18/CIFAR
                       on the plain per-layer path (one image), the serving
                       sweep (Poisson arrivals of a ResNet-18/ResNet-50 mix),
                       ResNet-18 224x224 at N = 16384, 4 primes, 64 images
                       as the batched graph, and the conventional (HRot/PMult)
                       convolution against this path on Table 9's layer shapes
  cpu_baseline         the CPU oracle (Algorithm 1 in C, OpenMP) on a sample,
                       all host threads and one thread
  client               the client-side steps around the step, timed apart:
                       online encryption (Algorithm 2) of every layer's input
                       against HBM bandwidth, and decryption of every layer's
                       extracted outputs (its NTTs against the butterfly peak)
  protocol             the x^2 + x protocol's server steps on every layer's
                       activation map, timed apart: PMult of the batch-encoded
                       a + r by 2r plus v (butterflies), and the combination
                       into [[a^2 + a]] (HBM bytes)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HBM_PEAK = 8.0e12                     # bytes/s, MI355X HBM3E
CUS, CLK = 256, 2.4e9                 # compute units, peak engine clock
# 32-bit lane-ops per clock per CU: add/sub/min, and integer multiply (mul_lo,
# mul_hi, mad_u64_u32). The valu_probe object checks them on the device.
SIMPLE_LANES, MUL_LANES = 128, 64
# The inverse NTT's butterfly as compiled (Gentleman-Sande with a Shoup
# twiddle, lazy [0, 2q)): 3 multiplier operations (mul_hi, then two
# mad_u64_u32 whose low word is the Shoup product, with no subtraction) + 5
# simple ops (sum, its conditional subtraction as sub + min, difference + 2q
# as add + sub).
BFLY_MULS, BFLY_SIMPLE = 3, 5
BFLY_PEAK = CUS * CLK / (BFLY_MULS / MUL_LANES + BFLY_SIMPLE / SIMPLE_LANES)
# MAC term: one v_mad_u64_u32.
MAC_PEAK = CUS * CLK * MUL_LANES


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--net", default="resnet50_224", choices=["resnet50_224", "resnet18_cifar", "resnet18_224"])
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--N", type=int, default=8192)
    ap.add_argument("--L", type=int, default=3)
    ap.add_argument("--t", type=int, default=2 ** 20)
    ap.add_argument("--plain-images", type=int, default=2)
    ap.add_argument("--cpu-fraction", type=float, default=1.0 / 16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-client", action="store_true",
                    help="skip the client-side (encrypt/decrypt) and activation-protocol timing")
    ap.add_argument("--t-batch", type=int, default=786433,
                    help="prime plaintext modulus = 1 mod 2N for the protocol's batch-encoded step")
    ap.add_argument("--seed", type=int, default=50)
    ap.add_argument("--stage-passes", type=int, default=3, help="eager passes timed per kernel for the roofline")
    ap.add_argument("--copy-gib", type=float, default=4.0, help="size of the HBM stream-copy calibration")
    ap.add_argument("--no-autotune", action="store_true", help="use the context's default launch shapes")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file: layers found there are not re-timed, new results are appended")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (ResNet-18/CIFAR plain, serving, ResNet-18 224 at N=16384)")
    ap.add_argument("--serve-rates", default="0.5,1.0", help="serving: offered load, fractions of saturation")
    ap.add_argument("--serve-duration", type=float, default=1.5, help="serving: seconds of arrivals per rate")
    ap.add_argument("--large-batch", type=int, default=64, help="ResNet-18 224x224 at N=16384: images per step")
    ap.add_argument("--large-steps", type=int, default=10)
    ap.add_argument("--no-probe", action="store_true", help="skip the register-only VALU probe")
    ap.add_argument("--no-conventional", action="store_true",
                    help="skip the conventional (HRot/PMult) convolution's Table 9 comparison")
    return ap.parse_args()


def hbm_copy(torch, dev, gib, reps=5):
    """Achievable HBM bandwidth: a plain device-to-device copy of `gib` GiB
    (read + write counted), timed with events on the current stream."""
    n = int(gib * 2 ** 30) // 4
    a = torch.empty(n, dtype=torch.int32, device=dev)
    b = torch.empty(n, dtype=torch.int32, device=dev)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 2 * n * 4, "ms": round(ms, 3), "GBps": round(2 * n * 4 / (ms * 1e-3) / 1e9, 1)}


# stage -> kernels launched for it (the MAC has register-tiled, LDS-staged and DMA-staged forms)
# (on layers whose MAC also carries out c0's transform, k_mac_c0x, the inverse
# NTT transforms c1 only and k_c0_finish adds the splits and the mask)
STAGE_KERNELS = {"ntt_fwd": ("k_ntt_fwd",), "mac": ("k_mac_tiled", "k_mac_lds", "k_mac_dma", "k_mac_c0x"),
                 "intt_mask_extract": ("k_intt_masked", "k_c0_finish")}


def measured_traffic(kernel: str, tag: str):
    """HBM bytes per launch of stage `kernel` (all kernels of the stage) from the
    committed rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE,
    copy-calibrated), or None when the summary is missing or was taken on a
    different kernel source."""
    from paper_2401_16732_amd.build import kernel_fingerprint
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", f"hbm_traffic_{tag}.md")
    if not os.path.exists(path):
        return None
    cur = kernel_fingerprint()
    got, val = None, None
    for line in open(path):
        if line.startswith("source_sha256_16:"):
            got = line.split(":", 1)[1].strip()
        elif line.startswith("traffic_bytes_per_launch:"):
            k, v = line.split(":", 1)[1].split("=")
            if k.strip() == f"stage {kernel}":
                val = float(v)
    return val if got == cur else None


def c0_in_mac(ly, B):
    """Whether the layer's shapes for B images have the MAC carry out c0's
    transform (mac_pre = 6)."""
    return hasattr(ly, "tuning") and ly.tuning(B)[1][9] == 6


def layer_counts(ly, B, N, L, c0_mac=None):
    """Algorithmic work of one layer on B images (no scratch round trips).
    Inverse-NTT butterflies are counted as full transforms of every output
    polynomial (c0's pruned stages included); where the MAC carries out c0's
    transform they are counted in the MAC stage (bfly_c0_mac), and the
    inverse NTT stage counts c1's only."""
    lay = ly.layout
    c_out = ly.shape[1]
    logn = int(math.log2(N))
    pin = B * lay.in_cts * 2 * L
    pout = B * lay.out_cts * 2 * L
    pc0 = pout // 2 if (c0_in_mac(ly, B) if c0_mac is None else c0_mac) else 0
    return {
        "bfly_fwd": pin * (N // 2) * logn,
        "bfly_inv": (pout - pc0) * (N // 2) * logn,
        "bfly_c0_mac": pc0 * (N // 2) * logn,
        "mac": B * lay.out_cts * lay.w_cts * 2 * L * N,
        "mask": B * c_out * lay.ho * lay.wo * L,
        # bytes each kernel must move through its interface
        "bytes_fwd": pin * N * 4 * 2,
        # (Yhat: c1 only where the MAC carries out c0's transform; its partial
        # sums, under 1% of those bytes, are left out)
        "bytes_mac": (c_out * lay.w_cts * L * N + B * lay.in_cts * 2 * L * N + (pout - pc0) * N) * 4,
        "bytes_inv": ((pout - pc0) * N + B * lay.out_cts * L * N + B * c_out * L * lay.ho * lay.wo
                      + B * c_out * lay.ho * lay.wo) * 4,
        # whole-path algorithmic bytes: weights once + inputs + c1 out + c0_ext out + mask
        "bytes_path": (B * (lay.in_cts * 2 * L * N + lay.out_cts * L * N + c_out * L * lay.ho * lay.wo
                            + c_out * lay.ho * lay.wo)) * 4,
        "bytes_w": c_out * lay.w_cts * L * N * 4,
    }


def client_pass(torch, dev, ctx, layers, ct_in, c0, c1, B, t, tg, passes=3, graphs=True):
    """Times the client-side entry points over every layer for B images:
    online encryption of the layer inputs (in place on ct_in, which stays a
    set of canonical ciphertexts) and decryption of the extracted outputs.
    graphs=False (profiling passes): one eager pass each, nothing timed."""
    N, L = ctx.N, ctx.L
    acts = [torch.randint(0, t, ly.act_shape(B), generator=tg, device=dev, dtype=torch.int32) for ly in layers]
    s = torch.randint(-1, 2, (N,), generator=tg, device=dev, dtype=torch.int64)
    sk = torch.stack([torch.remainder(s, q) for q in ctx.primes]).to(torch.int32).contiguous()
    ws = torch.empty((max(ly.decrypt_workspace_words(B) for ly in layers),), dtype=torch.int32, device=dev)
    m = torch.empty((max(math.prod(ly.mask_shape(B)) for ly in layers),), dtype=torch.int32, device=dev)

    def enc():
        for k, ly in enumerate(layers):
            ly.encrypt_online(acts[k], ct_in[k], ct_in[k], B)

    def dec():
        for k, ly in enumerate(layers):
            ly.decrypt_extracted(c0[k], c1[k], sk, m, B, ws)

    # each pass is recorded once as a graph and replayed, so that the host's
    # per-call cost (tens of microseconds, more than a small layer's kernel)
    # does not enter the device time
    res = {}
    for name, fn in (("encrypt_online", enc), ("decrypt_extracted", dec)):
        fn()
        torch.cuda.synchronize()
        if not graphs:
            continue
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            fn()
        graph.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(passes):
            graph.replay()
        e1.record()
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / passes
        del graph
    # encryption: read and write c0 of every input ciphertext, read the activations
    enc_bytes = sum(B * ly.layout.in_cts * L * N * 8 + math.prod(ly.act_shape(B)) * 4 for ly in layers)
    # decryption: forward and inverse NTT of every output ciphertext's c1
    dec_bfly = sum(2 * B * ly.layout.out_cts * L * (N // 2) * int(math.log2(N)) for ly in layers)
    if not graphs:
        return None, acts
    enc_s, dec_s = res["encrypt_online"] * 1e-3, res["decrypt_extracted"] * 1e-3
    return {
        "encrypt_online": {"ms_per_image": round(res["encrypt_online"] / B, 4), "launches": len(layers),
                           "algorithmic_bytes": enc_bytes, "achieved_GBps": round(enc_bytes / enc_s / 1e9, 1),
                           "hbm_frac": round(enc_bytes / enc_s / HBM_PEAK, 4)},
        "decrypt_extracted": {"ms_per_image": round(res["decrypt_extracted"] / B, 4), "launches": 3 * len(layers),
                              "butterflies": dec_bfly, "tbutterfly_per_s": round(dec_bfly / dec_s / 1e12, 4),
                              "alu_frac": round(dec_bfly / dec_s / BFLY_PEAK, 4)},
    }, acts


def protocol_pass(torch, dev, hconv, ctx, layers, ct_in, acts, B, tg, t_batch, passes=3, graphs=True):
    """Times the server steps of the x^2 + x protocol over every layer's
    activation map for B images. Step 1 (PMult of the batch-encoded a + r by
    2r, plus v) needs a prime plaintext modulus = 1 mod 2N: it runs on a second
    context with t = t_batch and the same primes, on B c_out ho wo slots per
    layer packed N to a ciphertext. Step 2 (the combination) runs on each
    layer's own input ciphertexts (x = ct_in, in place; y a buffer of its own)
    with that layer's activation-shaped r and v."""
    from paper_2401_16732_amd import workloads as W
    N, L = ctx.N, ctx.L
    cb = hconv.Context(N, L, t_batch, primes=ctx.primes)
    n_ct = [-(-(B * ly.shape[1] * ly.layout.ho * ly.layout.wo) // N) for ly in layers]
    mx = max(n_ct)
    ct_b = W.gen_ct_limbs_torch(tg, (mx, 2), ctx.primes, N, dev)
    r = torch.randint(0, t_batch, (mx, N), generator=tg, device=dev, dtype=torch.int32)
    v = torch.randint(0, t_batch, (mx, N), generator=tg, device=dev, dtype=torch.int32)
    out = torch.empty_like(ct_b)
    ws = torch.empty((cb.act_workspace_words(mx),), dtype=torch.int32, device=dev)

    def step1():
        for n in n_ct:
            cb.act_pmult(ct_b[:n], r[:n], v[:n], out[:n], ws)

    # y: canonical residues (below every prime) at addresses of their own
    ybuf = torch.randint(0, min(ctx.primes), (max(t_.numel() for t_ in ct_in),), generator=tg, device=dev,
                         dtype=torch.int32)
    ys = [ybuf[:t_.numel()].view(t_.shape) for t_ in ct_in]

    def step2():
        for k, ly in enumerate(layers):
            ly.act_combine(ct_in[k], ys[k], acts[k], acts[k], ct_in[k], B)

    res = {}
    for name, fn in (("act_pmult", step1), ("act_combine", step2)):
        fn()
        torch.cuda.synchronize()
        if not graphs:
            continue
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            fn()
        graph.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(passes):
            graph.replay()
        e1.record()
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / passes
        del graph
    cb.close()
    if not graphs:
        return None
    # step 1 per ciphertext: PMult of 2L polynomials (two transforms each), batch
    # encoding of r and v (one inverse transform mod t each), L forward transforms of 2r
    per_ct = (4 * L + 2 + L) * (N // 2) * int(math.log2(N))
    bfly = sum(n_ct) * per_ct
    # step 2: read x and y, write the result (2 L N words each per ciphertext), read r and v
    cbytes = sum(B * ly.layout.in_cts * 2 * L * N * 4 * 3 + 2 * math.prod(ly.act_shape(B)) * 4 for ly in layers)
    s1, s2 = res["act_pmult"] * 1e-3, res["act_combine"] * 1e-3
    return {
        "t_batch": t_batch, "ciphertexts_step1": sum(n_ct),
        "act_pmult": {"ms_per_image": round(res["act_pmult"] / B, 4), "butterflies": bfly,
                      "tbutterfly_per_s": round(bfly / s1 / 1e12, 4), "alu_frac": round(bfly / s1 / BFLY_PEAK, 4)},
        "act_combine": {"ms_per_image": round(res["act_combine"] / B, 4), "algorithmic_bytes": cbytes,
                        "achieved_GBps": round(cbytes / s2 / 1e9, 1), "hbm_frac": round(cbytes / s2 / HBM_PEAK, 4)},
    }


def cpu_baseline(specs, N, L, t, frac, seed, frac_single=None):
    """The oracle (Algorithm 1 in C, OpenMP) on every layer for one image over
    the first ceil(frac * c_out) output channels; Algorithm 1's work is the same
    for every output channel, so the time scales by c_out / sampled. Then the
    same on one thread over ceil(frac_single * c_out) channels."""
    import numpy as np
    from oracle import calg1, layout, params
    from paper_2401_16732_amd import workloads as W
    primes = params.rns_primes(N, L)

    def run(fr):
        g = W.rng(seed + 1)
        total_s, sampled, full = 0.0, 0, 0
        for spec in specs:
            P = layout.plan(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
            f = W.gen_filters(g, spec)
            x = W.gen_ct_limbs(g, (P.G, 2), primes, N)
            n = max(1, math.ceil(fr * spec.c_o))
            t0 = time.perf_counter()
            calg1.alg1_layer(x, f, P, primes, outputs=np.arange(n))
            dt = time.perf_counter() - t0
            total_s += dt * spec.c_o / n
            sampled += n
            full += spec.c_o
        return total_s, sampled, full

    threads = calg1.threads()
    total_s, sampled, full = run(frac)
    out = {"value": round(total_s * 1e3, 1), "unit": "ms/image", "cores": threads, "kind": "oracle",
           "sample": f"1 image, every layer, first {sampled} of {full} output channels "
                     f"(~{sampled / full:.4f} of the Algorithm 1 work), scaled by c_out/sampled per layer",
           "nproc": os.cpu_count(), "cpu_model": calg1.cpu_model(), "build": "gcc -O3 -march=native -fopenmp"}
    if frac_single:
        calg1.set_threads(1)
        try:
            s1, sampled1, _ = run(frac_single)
        finally:
            calg1.set_threads(threads)
        out["single_thread"] = {"value": round(s1 * 1e3, 1), "unit": "ms/image", "cores": 1,
                                "sample": f"first {sampled1} of {full} output channels, scaled the same way"}
    return out


def event_ms(torch, fn, reps):
    """Mean ms of fn() over reps back-to-back calls on the current stream
    (one untimed call first)."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def roofline_of(stage, tot, nlayers, bfly_peak, mac_peak):
    """The dominant kernel (largest eager stage time) against its ceiling."""
    names = [("ntt_fwd", stage[0], tot["bfly_fwd"], tot["bytes_fwd"]),
             ("mac", stage[1], tot["mac"], tot["bytes_mac"]),
             ("intt_mask_extract", stage[2], tot["bfly_inv"], tot["bytes_inv"])]
    kname, kms, kops, kbytes = max(names, key=lambda r: r[1])
    ops_peak = mac_peak if kname == "mac" else bfly_peak
    t_alu, t_hbm = kops / ops_peak, kbytes / HBM_PEAK
    if t_alu >= t_hbm:
        ach = kops / (kms * 1e-3)
        roof = {"bound": "alu", "achieved": round(ach / 1e12, 4), "peak": round(ops_peak / 1e12, 4),
                "unit": "Tmac/s" if kname == "mac" else "Tbutterfly/s"}
    else:
        ach = kbytes / (kms * 1e-3)
        roof = {"bound": "hbm", "achieved": round(ach / 1e9, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof["algorithmic_bytes_per_launch"] = round(kbytes / nlayers)
    roof["kernel"] = kname
    roof["launches"] = nlayers
    roof["ms_total"] = round(kms, 3)
    roof["algorithmic_ops"] = kops
    roof["algorithmic_bytes"] = kbytes
    roof["alu_frac"] = round(kops / (kms * 1e-3) / ops_peak, 4)
    roof["hbm_frac"] = round(kbytes / (kms * 1e-3) / HBM_PEAK, 4)
    return roof


def autotune_single(hconv, ctx, layers, ct_in, mask, c0, c1):
    """Autotune every layer for one image (the plain legs' batch size) on the
    first image of the given buffers; the layers keep their other tunings."""
    bt1 = hconv.Batch(ctx, layers, 1)
    bt1.autotune([x[:1] for x in ct_in], [m[:1] for m in mask], [v[:1] for v in c0], [v[:1] for v in c1])
    bt1.close()


def cfg_resnet18_cifar(torch, dev, hconv, W, a, ctx, probe_peaks):
    """ResNet-18/CIFAR at N = 8192, 3 primes, t = 2^20, one image, one launch
    sequence per layer (the plain per-layer path), launch shapes autotuned for
    one image. Returns the result object and the layers (kept for serving)."""
    N, L, t = ctx.N, ctx.L, ctx.t
    specs = W.resnet18_cifar()
    g = W.rng(a.seed + 18)
    layers = [hconv.Layer(ctx, s.c_i, s.c_o, s.h, s.w, s.f_w, s.stride, W.gen_filters(g, s)) for s in specs]
    tg = torch.Generator(device=dev)
    tg.manual_seed(a.seed + 18)
    B = 1
    ct_in = [W.gen_ct_limbs_torch(tg, ly.in_shape(B)[:3], ctx.primes, N, dev) for ly in layers]
    mask = [torch.randint(0, t, ly.mask_shape(B), generator=tg, device=dev, dtype=torch.int32) for ly in layers]
    c0 = [torch.empty(ly.c0_shape(B), dtype=torch.int32, device=dev) for ly in layers]
    c1 = [torch.empty(ly.c1_shape(B), dtype=torch.int32, device=dev) for ly in layers]
    autotune_single(hconv, ctx, layers, ct_in, mask, c0, c1)
    ws = torch.empty((max(ly.workspace_words(B, True) for ly in layers),), dtype=torch.int32, device=dev)

    def one_image():
        for k, ly in enumerate(layers):
            ly.conv_masked(ct_in[k], mask[k], c0[k], c1[k], B, ws)

    ms = event_ms(torch, one_image, 10)
    tot = {}
    for ly in layers:
        for k, v in layer_counts(ly, B, N, L).items():
            tot[k] = tot.get(k, 0) + v
    bfly, mac = tot["bfly_fwd"] + tot["bfly_inv"] + tot["bfly_c0_mac"], tot["mac"]
    sec = ms * 1e-3
    bytes_ = tot["bytes_path"] + tot["bytes_w"]
    res = {"workload": "resnet18_cifar HE convolution, 20 conv layers, one image, per-layer launches",
           "N": N, "L": L, "t": t, "batch": B, "layers": len(layers), "ms_per_image": round(ms, 4),
           "modmul_per_s": round((bfly + mac + tot["mask"]) / sec, 1),
           "alu_frac": round((bfly / probe_peaks[0] + mac / probe_peaks[1]) / sec, 4),
           "hbm_frac": round(bytes_ / sec / HBM_PEAK, 4), "path_bytes": bytes_}
    del ct_in, mask, c0, c1, ws
    return res, layers


def cfg_resnet18_224_large(torch, dev, hconv, W, a, probe_peaks):
    """ResNet-18 224x224 at N = 16384, 4 primes, t = 2^24, B images as the
    batched graph (mask add and extraction fused into the inverse NTT),
    autotuned; ms per image and the dominant kernel's roofline."""
    N, L, t, B = 16384, 4, 2 ** 24, a.large_batch
    ctx = hconv.Context(N, L, t)
    specs = W.resnet18_224()
    g = W.rng(a.seed + 224)
    t0 = time.perf_counter()
    layers = [hconv.Layer(ctx, s.c_i, s.c_o, s.h, s.w, s.f_w, s.stride, W.gen_filters(g, s)) for s in specs]
    torch.cuda.synchronize()
    enc_ms = (time.perf_counter() - t0) * 1e3
    tg = torch.Generator(device=dev)
    tg.manual_seed(a.seed + 224)
    ct_in = [W.gen_ct_limbs_torch(tg, ly.in_shape(B)[:3], ctx.primes, N, dev) for ly in layers]
    mask = [torch.randint(0, t, ly.mask_shape(B), generator=tg, device=dev, dtype=torch.int32) for ly in layers]
    c0 = [torch.empty(ly.c0_shape(B), dtype=torch.int32, device=dev) for ly in layers]
    c1 = [torch.empty(ly.c1_shape(B), dtype=torch.int32, device=dev) for ly in layers]
    bt = hconv.Batch(ctx, layers, B)
    t1 = time.perf_counter()
    bt.autotune(ct_in, mask, c0, c1)
    tune_ms = (time.perf_counter() - t1) * 1e3
    ms = event_ms(torch, lambda: bt.run(ct_in, mask, c0, c1), a.large_steps)
    acc = [0.0, 0.0, 0.0]
    for _ in range(max(1, a.stage_passes)):
        acc = [x + y for x, y in zip(acc, bt.run_timed(ct_in, mask, c0, c1))]
    stage = [x / max(1, a.stage_passes) for x in acc]
    tot = {}
    for ly in layers:
        for k, v in layer_counts(ly, B, N, L).items():
            tot[k] = tot.get(k, 0) + v
    bfly, mac = tot["bfly_fwd"] + tot["bfly_inv"] + tot["bfly_c0_mac"], tot["mac"]
    sec = ms * 1e-3
    roof = roofline_of(stage, tot, len(layers), probe_peaks[0], probe_peaks[1])
    res = {"workload": "resnet18_224 HE convolution, 20 conv layers, batched HIP graph",
           "N": N, "L": L, "primes": ctx.primes, "t": t, "batch": B, "layers": len(layers),
           "ms_per_step": round(ms, 3), "ms_per_image": round(ms / B, 4), "steps": a.large_steps,
           "weight_encode_ms": round(enc_ms, 1), "autotune_ms": round(tune_ms, 1), "mac_grid_cap": bt.mac_cap,
           "stage_ms_eager": [round(v, 3) for v in stage],
           "modmul_per_s": round((bfly + mac + tot["mask"]) / sec, 1),
           "alu_frac": round((bfly / probe_peaks[0] + mac / probe_peaks[1]) / sec, 4),
           "path_hbm_frac": round((tot["bytes_path"] + tot["bytes_w"]) / sec / HBM_PEAK, 4),
           "roofline": roof}
    bt.close()
    for ly in layers:
        ly.close()
    del ct_in, mask, c0, c1
    ctx.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


# Table 9 layer shapes (H x W, c_in, c_out, f) whose image fits one slot row at N = 8192
TABLE9 = [((64, 64), 64, 64, 3), ((64, 64), 3, 64, 7), ((56, 56), 256, 256, 3), ((32, 32), 16, 16, 3),
          ((32, 32), 128, 128, 3), ((28, 28), 512, 512, 3), ((16, 16), 64, 64, 3), ((16, 16), 256, 256, 3),
          ((8, 8), 128, 128, 3), ((8, 8), 512, 512, 3), ((4, 4), 512, 512, 3)]
# the paper's conventional / best-DRot time ratio for the same shapes (CPU, n = 2048)
TABLE9_PAPER_RATIO = [55.7, 29.4, 94.3, 92.7, 78.5, 93.5, 30.6, 33.3, 10.2, 12.6, 4.0]


def conventional_vs_drot(torch, dev, hconv, W, a):
    """The conventional convolution (batch encoding, HRot with 10-bit digit key
    switching, PMult) against this library's direct-encoding convolution on
    Table 9's layer shapes at N = 8192, 3 primes, t = 786433, one image: ms per
    layer and their ratio, next to the paper's CPU ratio."""
    N, L, t, T = 8192, 3, 786433, 10
    ctx = hconv.Context(N, L, t)
    rows = []
    g = W.rng(a.seed + 9)
    tg = torch.Generator(device=dev)
    tg.manual_seed(a.seed + 9)
    for ((h, w), ci, co, f), paper in zip(TABLE9, TABLE9_PAPER_RATIO):
        filt = g.integers(-128, 128, size=(co, ci, f, f)).astype("int8")
        cc = hconv.CConv(ctx, ci, co, h, w, f, filt, T)
        R, LD = cc.layout.rotations, cc.layout.digits
        s = torch.randint(-1, 2, (N,), generator=tg, device=dev, dtype=torch.int64)
        sk = torch.stack([torch.remainder(s, q) for q in ctx.primes]).to(torch.int32).contiguous()
        keys = torch.empty((cc.keys_words(),), dtype=torch.int32, device=dev)
        ka = W.gen_ct_limbs_torch(tg, (R * LD,), ctx.primes, N, dev)
        ke = torch.randint(-8, 9, (R * LD, N), generator=tg, device=dev, dtype=torch.int32)
        kws = torch.empty((cc.keygen_workspace_words(),), dtype=torch.int32, device=dev)
        cc.keygen(sk, ka, ke, keys, kws)
        del ka, ke, kws
        ct = W.gen_ct_limbs_torch(tg, (1, cc.layout.g_in, 2), ctx.primes, N, dev)
        out = torch.empty((1, cc.layout.g_out, 2, L, N), dtype=torch.int32, device=dev)
        ws = torch.empty((cc.workspace_words(1),), dtype=torch.int32, device=dev)
        conv_ms = event_ms(torch, lambda: cc.run(keys, ct, out, 1, ws), 3)
        del ct, out, ws, keys
        cc.close()
        ly = hconv.Layer(ctx, ci, co, h, w, f, 1, filt)
        x = W.gen_ct_limbs_torch(tg, ly.in_shape(1)[:3], ctx.primes, N, dev)
        m = torch.randint(0, t, ly.mask_shape(1), generator=tg, device=dev, dtype=torch.int32)
        c0 = torch.empty(ly.c0_shape(1), dtype=torch.int32, device=dev)
        c1 = torch.empty(ly.c1_shape(1), dtype=torch.int32, device=dev)
        lws = torch.empty((ly.workspace_words(1, True),), dtype=torch.int32, device=dev)
        drot_ms = event_ms(torch, lambda: ly.conv_masked(x, m, c0, c1, 1, lws), 5)
        if not ly.layout.tiled and ci * f * f <= 2 ** 17:
            drot_ms = min(drot_ms, event_ms(torch, lambda: ly.conv_masked_direct(x, m, c0, c1, 1), 5))
        ly.close()
        del x, m, c0, c1, lws
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        rows.append({"hw": [h, w], "c_in": ci, "c_out": co, "f": f, "rotations": R,
                     "conventional_ms": round(conv_ms, 4), "drot_ms": round(drot_ms, 4),
                     "ratio": round(conv_ms / drot_ms, 2), "paper_cpu_ratio": paper})
    ctx.close()
    return {"workload": "Table 9 layer shapes (h w <= N/2), one image, N=8192, 3 primes, t=786433, "
                        "10-bit digits; DRot path = the faster of the NTT path and the coefficient-domain conv",
            "rows": rows}


def main():
    a = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (each image is independent; "
              "see the design notes on sharding). Use --gpus 1.", file=sys.stderr)
        return 2
    import torch
    from paper_2401_16732_amd import hconv
    from paper_2401_16732_amd import serve as S
    from paper_2401_16732_amd import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log = lambda s: print(f"[bench] {s}", file=sys.stderr, flush=True)

    # register-only VALU rates of this device: the lane rates the ALU peaks assume
    probe = None
    if not a.no_probe:
        r = hconv.valu_probe(0)
        unit = CUS * CLK
        probe = {"simple_lanes_per_clk_cu": round(r["simple_ops_per_s"] / unit, 2),
                 "mul_lanes_per_clk_cu": round(r["mul_ops_per_s"] / unit, 2),
                 "mad64_lanes_per_clk_cu": round(r["mad64_ops_per_s"] / unit, 2),
                 "butterflies_per_s": round(r["butterflies_per_s"], 1),
                 "butterfly_frac_of_peak": round(r["butterflies_per_s"] / BFLY_PEAK, 4),
                 "mad64_per_s": round(r["mad64_ops_per_s"], 1),
                 "device_compute_units": r["compute_units"], "device_clock_hz": r["clock_hz"],
                 "measured_clock_hz": round(r["measured_clock_hz"], 1),
                 "assumed": {"simple_lanes_per_clk_cu": SIMPLE_LANES, "mul_lanes_per_clk_cu": MUL_LANES,
                             "butterfly": f"{BFLY_MULS} multiplies + {BFLY_SIMPLE} simple ops",
                             "bfly_peak": BFLY_PEAK, "mac_peak": MAC_PEAK}}
        log(f"VALU probe: clock {r['measured_clock_hz'] / 1e9:.3f} GHz; simple {probe['simple_lanes_per_clk_cu']} "
            f"mul {probe['mul_lanes_per_clk_cu']} "
            f"mad64 {probe['mad64_lanes_per_clk_cu']} lanes/clk/CU; butterflies {r['butterflies_per_s'] / 1e12:.3f} T/s "
            f"({probe['butterfly_frac_of_peak']:.3f} of {BFLY_PEAK / 1e12:.3f} T)")
    peaks = (BFLY_PEAK, MAC_PEAK)

    N, L, t, B = a.N, a.L, a.t, a.batch
    ctx = hconv.Context(N, L, t)
    specs = W.NETS[a.net]()
    g = W.rng(a.seed)

    # offline: resident NTT-domain weights (timed apart, like the paper's offline phase)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    layers = [hconv.Layer(ctx, s.c_i, s.c_o, s.h, s.w, s.f_w, s.stride, W.gen_filters(g, s)) for s in specs]
    torch.cuda.synchronize()
    encode_ms = (time.perf_counter() - t0) * 1e3
    log(f"{a.net}: {len(layers)} layers encoded in {encode_ms:.0f} ms")

    tg = torch.Generator(device=dev)
    tg.manual_seed(a.seed)
    ct_in = [W.gen_ct_limbs_torch(tg, ly.in_shape(B)[:3], ctx.primes, N, dev) for ly in layers]
    mask = [torch.randint(0, t, ly.mask_shape(B), generator=tg, device=dev, dtype=torch.int32) for ly in layers]
    c0 = [torch.empty(ly.c0_shape(B), dtype=torch.int32, device=dev) for ly in layers]
    c1 = [torch.empty(ly.c1_shape(B), dtype=torch.int32, device=dev) for ly in layers]
    bt = hconv.Batch(ctx, layers, B)
    torch.cuda.synchronize()
    log(f"inputs resident; batch workspace {bt.workspace_bytes / 2**30:.1f} GiB")
    tune_ms = None
    if not a.no_autotune:
        t1 = time.perf_counter()
        bt.autotune(ct_in, mask, c0, c1, cache_path=a.tune_cache)
        tune_ms = (time.perf_counter() - t1) * 1e3
        log(f"autotuned {len(layers)} layers in {tune_ms:.0f} ms; graph MAC grid cap {bt.mac_cap}")

    for _ in range(a.warmup):
        bt.run(ct_in, mask, c0, c1)
    torch.cuda.synchronize()
    ms_step = float("nan")
    spread = None
    if a.steps > 0:
        # one event between consecutive steps on the launch stream: the whole
        # region (first to last) gives ms_per_step, the gaps the per-step spread
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps + 1)]
        w0 = time.perf_counter()
        ev[0].record()
        for k in range(a.steps):
            bt.run(ct_in, mask, c0, c1)
            ev[k + 1].record()
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - w0) * 1e3 / a.steps
        ms_step = ev[0].elapsed_time(ev[-1]) / a.steps
        per = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(a.steps))
        q = lambda f: per[min(len(per) - 1, int(round(f * (len(per) - 1))))]
        spread = {"median": round(q(0.5), 3), "p10": round(q(0.1), 3), "p90": round(q(0.9), 3)}
        log(f"batched: {ms_step:.2f} ms/step ({ms_step / B:.3f} ms/image), wall {wall_ms:.2f}")

    # per-kernel stage times (eager, events around every launch on its stream)
    acc = [0.0, 0.0, 0.0]
    for _ in range(max(1, a.stage_passes)):
        st = bt.run_timed(ct_in, mask, c0, c1)
        acc = [x + y for x, y in zip(acc, st)]
    stage = [x / max(1, a.stage_passes) for x in acc]
    torch.cuda.synchronize()
    log(f"stages (eager, ms): fwd {stage[0]:.2f} mac {stage[1]:.2f} inv {stage[2]:.2f}")
    copy = hbm_copy(torch, dev, a.copy_gib)
    log(f"HBM copy: {copy['GBps']} GB/s")

    tot = {}
    for ly in layers:
        for k, v in layer_counts(ly, B, N, L).items():
            tot[k] = tot.get(k, 0) + v
    modmul = tot["bfly_fwd"] + tot["bfly_inv"] + tot["bfly_c0_mac"] + tot["mac"] + tot["mask"]

    # plain path: one launch sequence per layer, one image at a time, with
    # launch shapes autotuned for one image (the layers keep their B-image
    # shapes for the batched graph)
    plain_ms = plain_hybrid_ms = None
    direct = []
    if not a.no_plain:
        if not a.no_autotune:
            t1 = time.perf_counter()
            autotune_single(hconv, ctx, layers, ct_in, mask, c0, c1)
            log(f"autotuned {len(layers)} layers for one image in {(time.perf_counter() - t1) * 1e3:.0f} ms")
        wsw = max(ly.workspace_words(1, True) for ly in layers)
        ws = torch.empty((wsw,), dtype=torch.int32, device=dev)

        def one_image(b):
            for k, ly in enumerate(layers):
                ly.conv_masked(ct_in[k][b], mask[k][b], c0[k][b], c1[k][b], 1, ws)

        one_image(0)
        torch.cuda.synchronize()
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0.record()
        for b in range(a.plain_images):
            one_image(b % B)
        p1.record()
        torch.cuda.synchronize()
        plain_ms = p0.elapsed_time(p1) / a.plain_images
        log(f"plain: {plain_ms:.3f} ms/image")

        # the same plain path with Flash's coefficient-domain conv on the layers
        # where it is faster at one image: tried where c_n f^2 <= 4 (untiled),
        # kept where its events beat the NTT path's
        direct = []
        for k, ly in enumerate(layers):
            cand = not ly.layout.tiled and ly.layout.cn * ly.shape[4] ** 2 <= 4
            if cand:
                tn = event_ms(torch, lambda: ly.conv_masked(ct_in[k][0], mask[k][0], c0[k][0], c1[k][0], 1, ws), 5)
                td = event_ms(torch, lambda: ly.conv_masked_direct(ct_in[k][0], mask[k][0], c0[k][0], c1[k][0], 1), 5)
                if td < tn:
                    direct.append(k)

        def one_image_hybrid(b):
            for k, ly in enumerate(layers):
                if k in direct:
                    ly.conv_masked_direct(ct_in[k][b], mask[k][b], c0[k][b], c1[k][b], 1)
                else:
                    ly.conv_masked(ct_in[k][b], mask[k][b], c0[k][b], c1[k][b], 1, ws)

        one_image_hybrid(0)
        torch.cuda.synchronize()
        p0.record()
        for b in range(a.plain_images):
            one_image_hybrid(b % B)
        p1.record()
        torch.cuda.synchronize()
        plain_hybrid_ms = p0.elapsed_time(p1) / a.plain_images
        log(f"plain with the coefficient-domain conv on {len(direct)} layers: {plain_hybrid_ms:.3f} ms/image")
        del ws

    client = protocol = None
    if not a.no_client:
        client, acts = client_pass(torch, dev, ctx, layers, ct_in, c0, c1, B, t, tg, graphs=a.steps > 0)
        protocol = protocol_pass(torch, dev, hconv, ctx, layers, ct_in, acts, B, tg, a.t_batch,
                                 graphs=a.steps > 0)
        del acts
    if protocol is not None:
        log(f"protocol: step 1 {protocol['act_pmult']['ms_per_image']:.3f} ms/image "
            f"({protocol['act_pmult']['tbutterfly_per_s']} T butterflies/s), step 2 "
            f"{protocol['act_combine']['ms_per_image']:.3f} ms/image ({protocol['act_combine']['achieved_GBps']} GB/s)")
    if client is not None:
        log(f"client: encrypt {client['encrypt_online']['ms_per_image']:.3f} ms/image "
            f"({client['encrypt_online']['achieved_GBps']} GB/s), decrypt "
            f"{client['decrypt_extracted']['ms_per_image']:.3f} ms/image")

    # roofline of the dominant kernel (largest stage time)
    roof = roofline_of(stage, tot, len(layers), *peaks)
    traffic = measured_traffic(roof["kernel"], f"resnet50_b{B}") if a.net == "resnet50_224" else None
    roof["traffic"] = None if traffic is None else round(traffic)
    roof["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    if probe is not None:
        kpeak = probe["mad64_per_s"] if roof["kernel"] == "mac" else probe["butterflies_per_s"]
        ach = roof["algorithmic_ops"] / (roof["ms_total"] * 1e-3)
        roof["frac_of_probe"] = round(ach / kpeak, 4)
    whole_alu = ((tot["bfly_fwd"] + tot["bfly_inv"] + tot["bfly_c0_mac"]) / peaks[0] + tot["mac"] / peaks[1]) / (ms_step * 1e-3)

    mac_cap = bt.mac_cap
    # the other workloads, after the headline's buffers are released
    configs = None
    if not a.no_configs and a.steps > 0 and a.net == "resnet50_224":
        bt.close()
        del ct_in, mask, c0, c1
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        configs = {}
        r18, r18_layers = cfg_resnet18_cifar(torch, dev, hconv, W, a, ctx, peaks)
        configs["resnet18_cifar_plain"] = r18
        log(f"resnet18_cifar plain: {r18['ms_per_image']:.3f} ms/image")
        sv = S.sweep(hconv, W, ctx, {"resnet18_cifar": r18_layers, "resnet50_224": layers}, mix=0.5,
                     rates=[float(v) for v in a.serve_rates.split(",")], duration=a.serve_duration,
                     arena_gib=128.0, max_batch=16, streams=4, max_inflight=8, burst=64, sets=2, seed=a.seed,
                     bfly_peak=peaks[0], mac_peak=peaks[1])
        sv["workload"] = ("serving: Poisson arrivals, 50% ResNet-50 224x224 / 50% ResNet-18 32x32 requests, "
                          "N=8192, 3 primes, continuous batching")
        configs["serving"] = sv
        log(f"serving: saturation {sv['saturation']['requests_per_s']} req/s; " + ", ".join(
            f"{r['rate_fraction']}x: p50 {r['p50_ms']} p99 {r['p99_ms']} ms" for r in sv["rates"]))
        for ly in r18_layers + layers:
            ly.close()
        layers = []
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        big = cfg_resnet18_224_large(torch, dev, hconv, W, a, peaks)
        configs["resnet18_224_n16384"] = big
        log(f"resnet18_224 N=16384 B={big['batch']}: {big['ms_per_image']:.3f} ms/image, "
            f"{big['roofline']['kernel']} {big['roofline']['frac']}")
        if not a.no_conventional:
            cv = conventional_vs_drot(torch, dev, hconv, W, a)
            configs["conventional_vs_drot"] = cv
            log("conventional / DRot path: " + ", ".join(
                f"{r['hw'][0]}^2 {r['c_in']}->{r['c_out']} {r['ratio']}x" for r in cv["rows"]))

    cpu = None
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(specs, N, L, t, a.cpu_fraction, a.seed, frac_single=a.cpu_fraction / 16)

    per_img = ms_step / B
    if a.steps == 0:
        print(json.dumps({"profile_pass": True, "stage_ms_eager": stage, "hbm_copy": copy}), flush=True)
        return 0
    best_plain = min(v for v in (plain_ms, plain_hybrid_ms) if v is not None) if plain_ms is not None else None
    out = {
        "metric": "HE-conv ms per ResNet-50 image + NTT modmul/s vs roofline, batched vs plain",
        "value": round(per_img, 4),
        "unit": "ms/image",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 3),
        "ms_per_step_spread": spread,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{a.net} HE convolution, all {len(specs)} conv layers, batched HIP graph",
                   "N": N, "L": L, "primes": ctx.primes, "t": t, "batch": B, "layers": len(specs),
                   "parallelism": "single GPU"},
        "images_per_s": round(1e3 / per_img, 2),
        "modmul_per_s": round(modmul / (ms_step * 1e-3), 1),
        "whole_step_alu_frac": round(whole_alu, 4),
        "plain_ms_per_image": None if plain_ms is None else round(plain_ms, 4),
        "plain_hybrid_ms_per_image": None if plain_hybrid_ms is None else round(plain_hybrid_ms, 4),
        "plain_hybrid_direct_layers": direct,
        "speedup_vs_plain": None if best_plain is None else round(best_plain / per_img, 3),
        "speedup_vs_plain_ntt_only": None if plain_ms is None else round(plain_ms / per_img, 3),
        "weight_encode_ms": round(encode_ms, 1),
        "autotune_ms": None if tune_ms is None else round(tune_ms, 1),
        "mac_grid_cap": mac_cap,
        "stage_ms_eager": [round(v, 3) for v in stage],
        "path_bytes_per_step": tot["bytes_path"] + tot["bytes_w"],
        "path_hbm_frac": round((tot["bytes_path"] + tot["bytes_w"]) / (ms_step * 1e-3) / HBM_PEAK, 4),
        "hbm_copy": copy,
        "valu_probe": probe,
        "roofline": roof,
        "cpu_baseline": cpu,
        "client": client,
        "protocol": protocol,
        "configs": configs,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
