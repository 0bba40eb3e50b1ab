"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (all 53 ResNet-50 layers, 16 images, autotuned launch shapes, one HIP
graph), and at the large ring (ResNet-18 224x224, N = 16384, 4 primes, 64
images, autotuned): every output of every layer of several images through a
Freivalds combination over output channels against the oracle, sampled outputs
against the oracle's closed form (bit-exact), and graph replays against eager
runs."""
import numpy as np
import pytest

from oracle import layout
from paper_2401_16732_amd import workloads as W

from gpu_util import check_layer_points, freivalds_check, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_16732_amd import hconv
    hconv.load()
    return hconv


def _net_batch(hc, net, N, L, t, B, seed):
    import torch
    ctx = hc.Context(N, L, t)
    specs = W.NETS[net]()
    g = W.rng(seed)
    filters = [W.gen_filters(g, s) for s in specs]
    layers = [hc.Layer(ctx, s.c_i, s.c_o, s.h, s.w, s.f_w, s.stride, f) for s, f in zip(specs, filters)]
    tg = torch.Generator(device="cuda")
    tg.manual_seed(seed)
    ct_in = [W.gen_ct_limbs_torch(tg, ly.in_shape(B)[:3], ctx.primes, N, "cuda") for ly in layers]
    mask = [torch.randint(0, t, ly.mask_shape(B), generator=tg, device="cuda", dtype=torch.int32) for ly in layers]
    c0 = [torch.zeros(ly.c0_shape(B), dtype=torch.int32, device="cuda") for ly in layers]
    c1 = [torch.zeros(ly.c1_shape(B), dtype=torch.int32, device="cuda") for ly in layers]
    return ctx, specs, filters, layers, ct_in, mask, c0, c1


def _check_net(ctx, specs, filters, ct_in, mask, c0, c1, images, t, g, npts):
    """Every output of each image in `images` (Freivalds over output channels)
    and npts sampled outputs by the closed form, for every layer."""
    for k, (s, f) in enumerate(zip(specs, filters)):
        P = layout.plan(ctx.N, s.c_i, s.c_o, s.h, s.w, s.f_w, s.stride)
        for b in images:
            print(f"  layer {k} {s.name} image {b}", flush=True)
            x = host(ct_in[k][b])
            freivalds_check(P, ctx.primes, ctx.delta_mod_q, t, x, f, mask[k][b], c0[k][b], c1[k][b], g)
            check_layer_points(P, ctx.primes, t, x, f, host(mask[k][b]), host(c0[k][b]), host(c1[k][b]), g,
                               npts=npts)


def _tuned_shapes(layers, B):
    """Every layer carries an autotuned shape set for this batch size."""
    for ly in layers:
        tb, tv = ly.tuning()
        assert tb == B, (tb, tv)


def _free(*objs):
    import torch
    for o in objs:
        if isinstance(o, list):
            for x in o:
                if hasattr(x, "close"):
                    x.close()
        elif hasattr(o, "close"):
            o.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_resnet50_batch16_graph_matches_oracle(hc):
    """The benchmark's configuration: ResNet-50 at B = 16, autotuned like
    bench.py, replayed as the graph; every output of images 0, 7 and 15."""
    import torch
    N, L, t, B = 8192, 3, 2 ** 20, 16
    print("resnet50_224 B=16 graph, autotuned", flush=True)
    ctx, specs, filters, layers, ct_in, mask, c0, c1 = _net_batch(hc, "resnet50_224", N, L, t, B, 50)
    bt = hc.Batch(ctx, layers, B)
    bt.autotune(ct_in, mask, c0, c1)
    _tuned_shapes(layers, B)
    for v in c0 + c1:
        v.zero_()
    bt.run(ct_in, mask, c0, c1)
    torch.cuda.synchronize()
    _check_net(ctx, specs, filters, ct_in, mask, c0, c1, (0, 7, B - 1), t, W.rng(7), npts=8)
    del ct_in, mask, c0, c1
    _free(bt, layers)


def test_graph_replays_match_eager(hc):
    """Replay the recorded graph several times with eager work and syncs in
    between; every replay must equal the eager (stream-ordered) result."""
    import torch
    N, L, t, B = 8192, 3, 2 ** 20, 16
    ctx = hc.Context(N, L, t)
    specs = [s for s in W.resnet50_224() if s.name in ("stem", "s1.b0.c2", "s2.b0.proj", "s3.b1.c1", "s4.b0.c3",
                                                         "s4.b2.c2")]
    g = W.rng(3)
    layers = [hc.Layer(ctx, s.c_i, s.c_o, s.h, s.w, s.f_w, s.stride, W.gen_filters(g, s)) for s in specs]
    tg = torch.Generator(device="cuda")
    tg.manual_seed(3)
    ct_in = [W.gen_ct_limbs_torch(tg, ly.in_shape(B)[:3], ctx.primes, N, "cuda") for ly in layers]
    mask = [torch.randint(0, t, ly.mask_shape(B), generator=tg, device="cuda", dtype=torch.int32) for ly in layers]
    outs = lambda: ([torch.zeros(ly.c0_shape(B), dtype=torch.int32, device="cuda") for ly in layers],
                    [torch.zeros(ly.c1_shape(B), dtype=torch.int32, device="cuda") for ly in layers])
    bt = hc.Batch(ctx, layers, B)
    e0, e1 = outs()
    bt.run_eager(ct_in, mask, e0, e1)
    torch.cuda.synchronize()
    g0, g1 = outs()
    x0, x1 = outs()
    for rep in range(3):
        print(f"graph replay {rep}", flush=True)
        for v in g0 + g1:
            v.zero_()
        bt.run(ct_in, mask, g0, g1)
        bt.run_eager(ct_in, mask, x0, x1)  # eager work between replays
        torch.cuda.synchronize()
        for k in range(len(layers)):
            assert torch.equal(g0[k], e0[k]) and torch.equal(g1[k], e1[k]), (rep, k)
            assert torch.equal(x0[k], e0[k]) and torch.equal(x1[k], e1[k]), (rep, k)
    del ct_in, mask, e0, e1, g0, g1, x0, x1
    _free(bt, layers)


def test_resnet18_224_large_ring_batch64_matches_oracle(hc):
    import torch
    N, L, t, B = 16384, 4, 2 ** 24, 64
    print("resnet18_224 N=16384 L=4 B=64 graph, autotuned", flush=True)
    ctx, specs, filters, layers, ct_in, mask, c0, c1 = _net_batch(hc, "resnet18_224", N, L, t, B, 18)
    bt = hc.Batch(ctx, layers, B)
    bt.autotune(ct_in, mask, c0, c1)
    _tuned_shapes(layers, B)
    for v in c0 + c1:
        v.zero_()
    bt.run(ct_in, mask, c0, c1)
    torch.cuda.synchronize()
    _check_net(ctx, specs, filters, ct_in, mask, c0, c1, (0, 37, B - 1), t, W.rng(8), npts=8)
    del ct_in, mask, c0, c1
    _free(bt, layers)


def test_autotuner_keeps_results_and_caches(hc, tmp_path):
    import torch
    N, L, t, B = 8192, 3, 2 ** 20, 16
    ctx = hc.Context(N, L, t)
    specs = [s for s in W.resnet50_224() if s.name in ("s1.b0.c2", "s3.b1.c1", "s4.b0.c3")]
    g = W.rng(5)
    layers = [hc.Layer(ctx, s.c_i, s.c_o, s.h, s.w, s.f_w, s.stride, W.gen_filters(g, s)) for s in specs]
    tg = torch.Generator(device="cuda")
    tg.manual_seed(5)
    ct_in = [W.gen_ct_limbs_torch(tg, ly.in_shape(B)[:3], ctx.primes, N, "cuda") for ly in layers]
    mask = [torch.randint(0, t, ly.mask_shape(B), generator=tg, device="cuda", dtype=torch.int32) for ly in layers]
    outs = lambda: ([torch.zeros(ly.c0_shape(B), dtype=torch.int32, device="cuda") for ly in layers],
                    [torch.zeros(ly.c1_shape(B), dtype=torch.int32, device="cuda") for ly in layers])
    bt = hc.Batch(ctx, layers, B)
    r0, r1 = outs()
    bt.run(ct_in, mask, r0, r1)
    cache = tmp_path / "tune.txt"
    s0, s1 = outs()
    print("autotune (timing)", flush=True)
    bt.autotune(ct_in, mask, s0, s1, cache_path=cache)
    tuned = [ly.tuning() for ly in layers]
    # every shape field set (mac_lds and mac_pre may legitimately be 0)
    assert all(tb == B and all(tv[i] > 0 for i in (0, 1, 2, 3, 4, 5, 6, 8)) for tb, tv in tuned), tuned
    assert len(cache.read_text().strip().splitlines()) == len(layers)
    a0, a1 = outs()
    bt.run(ct_in, mask, a0, a1)  # graph re-recorded with the tuned shapes
    torch.cuda.synchronize()
    for k in range(len(layers)):
        assert torch.equal(a0[k], r0[k]) and torch.equal(a1[k], r1[k]), k
    for ly in layers:
        ly.clear_tuning()
        assert ly.tuning()[0] == 0
    print("autotune (cache)", flush=True)
    bt.autotune(ct_in, mask, s0, s1, cache_path=cache)
    assert [ly.tuning() for ly in layers] == tuned
    assert len(cache.read_text().strip().splitlines()) == len(layers)  # nothing re-timed
    del ct_in, mask, r0, r1, s0, s1, a0, a1
    _free(bt, layers)
