"""The batch as a two-stream pipeline over output-channel chunks
(hc_batch_run_pipelined) gives the graph's outputs bit for bit: ResNet-50
layers at B = 16 (tiled stem, stride-2 and 1x1 layers) with small chunks, so
that many chunks rotate through 2 or 3 buffers across layer boundaries, and
ResNet-18 224x224 layers at N = 16384 with B = 64 (more images than one
inverse-NTT launch takes per chunk). The batch graph with a grid cap on its
MAC launches gives the same outputs as without, for every DMA-staged MAC tile
also on ragged tiles and short reductions."""
import pytest

from paper_2401_16732_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_16732_amd import hconv
    hconv.load()
    return hconv


def _case(hc, net, names, N, L, t, B, seed):
    import torch
    ctx = hc.Context(N, L, t)
    specs = [s for s in W.NETS[net]() if s.name in names]
    g = W.rng(seed)
    layers = [hc.Layer(ctx, s.c_i, s.c_o, s.h, s.w, s.f_w, s.stride, W.gen_filters(g, s)) for s in specs]
    tg = torch.Generator(device="cuda")
    tg.manual_seed(seed)
    ct_in = [W.gen_ct_limbs_torch(tg, ly.in_shape(B)[:3], ctx.primes, N, "cuda") for ly in layers]
    mask = [torch.randint(0, t, ly.mask_shape(B), generator=tg, device="cuda", dtype=torch.int32) for ly in layers]
    outs = lambda: ([torch.zeros(ly.c0_shape(B), dtype=torch.int32, device="cuda") for ly in layers],
                    [torch.zeros(ly.c1_shape(B), dtype=torch.int32, device="cuda") for ly in layers])
    return ctx, layers, ct_in, mask, outs


@pytest.mark.parametrize("chunk_mib,nbuf", [(8, 2), (20, 3)])
def test_pipelined_equals_graph_resnet50(hc, chunk_mib, nbuf):
    import torch
    N, L, t, B = 8192, 3, 2 ** 20, 16
    ctx, layers, ct_in, mask, outs = _case(hc, "resnet50_224", ("stem", "s1.b0.c2", "s2.b0.c2", "s2.b0.proj",
                                                                 "s3.b1.c1", "s4.b0.c3"), N, L, t, B, 61)
    bt = hc.Batch(ctx, layers, B)
    g0, g1 = outs()
    bt.run(ct_in, mask, g0, g1)
    for rep in range(2):
        print(f"pipelined chunk {chunk_mib} MiB x{nbuf}, run {rep}", flush=True)
        p0, p1 = outs()
        bt.run_pipelined(ct_in, mask, p0, p1, chunk_bytes=chunk_mib << 20, nbuf=nbuf)
        torch.cuda.synchronize()
        for k in range(len(layers)):
            assert torch.equal(p0[k], g0[k]) and torch.equal(p1[k], g1[k]), (rep, k)
    bt.close()
    for ly in layers:
        ly.close()


def test_pipelined_equals_graph_large_ring_b64(hc):
    import torch
    N, L, t, B = 16384, 4, 2 ** 24, 64
    ctx, layers, ct_in, mask, outs = _case(hc, "resnet18_224", ("stem", "s2.b1.c1", "s4.b2.c2"), N, L, t, B, 62)
    bt = hc.Batch(ctx, layers, B)
    g0, g1 = outs()
    bt.run(ct_in, mask, g0, g1)
    print("pipelined N=16384 B=64", flush=True)
    p0, p1 = outs()
    bt.run_pipelined(ct_in, mask, p0, p1, chunk_bytes=96 << 20, nbuf=3)
    torch.cuda.synchronize()
    for k in range(len(layers)):
        assert torch.equal(p0[k], g0[k]) and torch.equal(p1[k], g1[k]), k
    bt.close()
    for ly in layers:
        ly.close()


@pytest.mark.parametrize("tile", [(4, 8, 2, 2, 4, 2), (2, 8, 4, 2, 4, 2)])
def test_mac_grid_cap_equals_uncapped(hc, tile):
    """The batch graph with its DMA-staged MAC launches capped (workgroups that
    loop over the tiles; 8 workgroups take hundreds of tiles each, 13 rounds
    down to 8, 264 is not a power of two, and 4 per compute unit) gives the
    uncapped graph's outputs (a new batch's default). One batch per cap, each
    recording its graph once."""
    import torch
    N, L, t, B = 8192, 3, 2 ** 20, 16
    ctx, layers, ct_in, mask, outs = _case(hc, "resnet50_224", ("stem", "s1.b0.c2", "s2.b0.proj", "s4.b0.c3"),
                                           N, L, t, B, 67)
    ctx.set_tuning(0, 0, *tile)
    ref = hc.Batch(ctx, layers, B)
    assert ref.mac_cap == 0
    g0, g1 = outs()
    ref.run(ct_in, mask, g0, g1)
    torch.cuda.synchronize()
    ref.close()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for cap in (8, 13, 264, 4 * cus):
        print(f"MAC tile {tile}, grid cap {cap}", flush=True)
        bt = hc.Batch(ctx, layers, B)
        bt.mac_cap = cap
        assert bt.mac_cap == cap
        p0, p1 = outs()
        bt.run(ct_in, mask, p0, p1)
        torch.cuda.synchronize()
        for k in range(len(layers)):
            assert torch.equal(p0[k], g0[k]) and torch.equal(p1[k], g1[k]), (cap, k)
        with pytest.raises(hc.HcError):
            bt.mac_cap = 5
        bt.close()
    for ly in layers:
        ly.close()


DMA_TILES = [(4, 8, 2, 2, 3, 2), (4, 8, 2, 2, 4, 2), (4, 8, 2, 2, 6, 2), (4, 8, 4, 2, 3, 2), (4, 8, 4, 2, 4, 2),
             (2, 8, 4, 2, 4, 2), (4, 4, 4, 2, 4, 2), (2, 8, 2, 2, 4, 2), (4, 4, 2, 2, 4, 2)]


@pytest.mark.parametrize("cap", [8, 64, 0])
def test_dma_mac_tile_loop_ragged(hc, cap):
    """Every DMA-staged MAC tile without epilogue stages, its workgroups
    looping over many tiles (caps 8 and 64) or taking one each (0), on layers
    whose tiles are ragged in both directions (20 output channels, 5 images)
    and whose reductions take 1, 2, 3, 5 and 6 input ciphertexts (fewer steps
    than the staging depth, as many, and more). The outputs equal the
    register-tiled MAC's (no LDS, uncapped)."""
    import torch
    N, L, t, B = 8192, 3, 2 ** 20, 5
    ctx = hc.Context(N, L, t)
    # 3x3 on 16x16: 25 channels per ciphertext, so c_i = 20, 30, 60, 110, 130
    # gives 1, 2, 3, 5, 6 input ciphertexts
    specs = [W.ConvSpec(ci, 20, 16, 16, 3, 1) for ci in (20, 30, 60, 110, 130)]
    g = W.rng(68)
    layers = [hc.Layer(ctx, s.c_i, s.c_o, s.h, s.w, s.f_w, s.stride, W.gen_filters(g, s)) for s in specs]
    assert [ly.layout.w_cts for ly in layers] == [1, 2, 3, 5, 6]
    tg = torch.Generator(device="cuda")
    tg.manual_seed(68)
    ct_in = [W.gen_ct_limbs_torch(tg, ly.in_shape(B)[:3], ctx.primes, N, "cuda") for ly in layers]
    mask = [torch.randint(0, t, ly.mask_shape(B), generator=tg, device="cuda", dtype=torch.int32) for ly in layers]
    outs = lambda: ([torch.zeros(ly.c0_shape(B), dtype=torch.int32, device="cuda") for ly in layers],
                    [torch.zeros(ly.c1_shape(B), dtype=torch.int32, device="cuda") for ly in layers])
    ctx.set_tuning(0, 0, 4, 4, 1, 4, 2, 0)
    ref = hc.Batch(ctx, layers, B)
    g0, g1 = outs()
    ref.run(ct_in, mask, g0, g1)
    torch.cuda.synchronize()
    ref.close()
    for tile in DMA_TILES:
        print(f"DMA MAC tile {tile}, grid cap {cap}", flush=True)
        ctx.set_tuning(0, 0, *tile)
        bt = hc.Batch(ctx, layers, B)
        bt.mac_cap = cap
        p0, p1 = outs()
        bt.run(ct_in, mask, p0, p1)
        torch.cuda.synchronize()
        for k in range(len(layers)):
            assert torch.equal(p0[k], g0[k]) and torch.equal(p1[k], g1[k]), (tile, cap, k)
        bt.close()
    for ly in layers:
        ly.close()


def test_c0_transform_in_mac_graph_eager_pipelined(hc):
    """ResNet-50's 7x7 layers (1x1 and 3x3, one with client subsampling) with
    the MAC tiles that carry out c0's transform: the batch graph, the eager run
    and the two-stream pipeline over channel chunks (each chunk its own split
    count) give the outputs of the plain tiles."""
    import torch
    N, L, t, B = 8192, 3, 2 ** 20, 16
    ctx, layers, ct_in, mask, outs = _case(hc, "resnet50_224", ("s4.b0.proj", "s4.b1.c1", "s4.b1.c2", "s4.b1.c3"),
                                           N, L, t, B, 69)
    ctx.set_tuning(0, 0, 4, 8, 2, 2, 4, 2, 0, 0)
    ref = hc.Batch(ctx, layers, B)
    g0, g1 = outs()
    ref.run(ct_in, mask, g0, g1)
    torch.cuda.synchronize()
    ref.close()
    for tile in ((4, 8, 2, 2, 4, 2), (4, 8, 4, 2, 3, 2)):
        ctx.set_tuning(0, 0, *tile, 0, 6)
        bt = hc.Batch(ctx, layers, B)
        for mode in ("graph", "eager", "pipelined 24 MiB x3"):
            print(f"c0 in the MAC, tile {tile}, {mode}", flush=True)
            p0, p1 = outs()
            if mode == "graph":
                bt.run(ct_in, mask, p0, p1)
            elif mode == "eager":
                bt.run_eager(ct_in, mask, p0, p1)
            else:
                bt.run_pipelined(ct_in, mask, p0, p1, chunk_bytes=24 << 20, nbuf=3)
            torch.cuda.synchronize()
            for k in range(len(layers)):
                assert torch.equal(p0[k], g0[k]) and torch.equal(p1[k], g1[k]), (tile, mode, k)
        bt.close()
    for ly in layers:
        ly.close()
