"""Serving loop: a request's results are the same alone and in a mix of other
requests and networks (tolerance 0), admission respects the HBM arena, and
the served outputs match the CPU oracle."""
import numpy as np
import pytest

from oracle import layout, params
from paper_2401_16732_amd import workloads as W

from gpu_util import check_layer_points, dev, host

pytestmark = pytest.mark.gpu

N, L, T = 8192, 3, 2 ** 20

# network a: the first ResNet-18/CIFAR layers plus a 1x1 layer at 56 x 56 (c_n = 2, so a
# group of one image takes the coefficient-domain conv and a larger group the NTT path)
NET_A_EXTRA = [W.ConvSpec(8, 16, 56, 56, 1, 1, "a.1x1")]

NET_B = [  # a small second network with other shapes: tiled 7x7/2 stem, 1x1/2, 5x5
    W.ConvSpec(3, 8, 64, 64, 7, 2, "b.stem"),
    W.ConvSpec(8, 16, 32, 32, 1, 2, "b.proj"),
    W.ConvSpec(8, 12, 16, 16, 5, 1, "b.c5"),
]


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_16732_amd import hconv
    ctx = hconv.Context(N, L, T)
    g = W.rng(99)
    nets = {}
    for name, specs in (("a", W.resnet18_cifar()[:6] + NET_A_EXTRA), ("b", NET_B)):
        filt = [W.gen_filters(g, s) for s in specs]
        layers = [hconv.Layer(ctx, s.c_i, s.c_o, s.h, s.w, s.f_w, s.stride, f) for s, f in zip(specs, filt)]
        nets[name] = (specs, filt, layers)
    return hconv, ctx, nets, g


def _inputs(ctx, specs, layers, g):
    xs, ms = [], []
    for s, ly in zip(specs, layers):
        lay = ly.layout
        xs.append(W.gen_ct_limbs(g, (lay.in_cts, 2), ctx.primes, N))
        ms.append(W.gen_mask(g, (s.c_o, lay.ho, lay.wo), T))
    return xs, ms


def _run(srv, plan, lockstep=False):
    """plan: list of (submit_at_step, net_id, ct_in, mask). Returns {index: request id}.
    lockstep: wait for the server's streams after every step, so that requests
    admitted in one step are ready together and every launched group finishes
    before the next step (groups then never split)."""
    ids = {}
    done = set()
    step = 0
    while len(done) < len(plan):
        for k, (at, net, x, m) in enumerate(plan):
            if at == step:
                ids[k] = srv.submit(net, x, m)
        srv.step()
        if lockstep:
            srv.sync()
        done.update(srv.poll())
        step += 1
        assert step < 100000, "server made no progress"
    return ids


def test_request_alone_equals_request_in_mix(setup):
    hconv, ctx, nets, g = setup
    import torch
    specs_a, filt_a, layers_a = nets["a"]
    specs_b, filt_b, layers_b = nets["b"]
    xa, ma = _inputs(ctx, specs_a, layers_a, g)
    dxa, dma = [dev(x) for x in xa], [dev(m) for m in ma]
    # alone
    print("serving: request alone", flush=True)
    srv = hconv.Server(ctx, arena_bytes=8 << 30, max_batch=16, streams=2)
    na, nb = srv.add_net(layers_a), srv.add_net(layers_b)
    rid = _run(srv, [(0, na, dxa, dma)])[0]
    # alone, its 1x1 layer at 56 x 56 (c_n f^2 = 2) ran through the coefficient-domain conv
    assert srv.stats()["direct_groups"] == 1, srv.stats()
    alone = [srv.outputs(rid, k, na) for k in range(len(layers_a))]
    alone = [(host(c0).copy(), host(c1).copy()) for c0, c1 in alone]
    srv.release(rid)
    srv.close()
    # in a mix: five other requests of network a are submitted in the same step as
    # it (so all six go through every layer as one group: the 1x1 layer takes the
    # NTT path), and requests of network b arrive before, with and after it
    print("serving: request in a mix", flush=True)
    plan = []
    others = []
    for k in range(9):
        net, specs, layers = (na, specs_a, layers_a) if k % 3 else (nb, specs_b, layers_b)
        x, m = _inputs(ctx, specs, layers, g)
        others.append((net, [dev(v) for v in x], [dev(v) for v in m]))
        plan.append((1 if net == na else k // 2, net, others[-1][1], others[-1][2]))
    plan.insert(4, (1, na, dxa, dma))
    srv = hconv.Server(ctx, arena_bytes=8 << 30, max_batch=16, streams=3, max_inflight=3)
    assert srv.add_net(layers_a) == na and srv.add_net(layers_b) == nb
    ids = _run(srv, plan, lockstep=True)
    st = srv.stats()
    assert st["completed"] == len(plan) and st["groups"] < st["images"], st  # some layers were batched
    # no group of network a had one image: the request's 1x1 layer ran in a group, by the NTT
    # path, and network b has no layer that takes the coefficient-domain conv
    assert st["direct_groups"] == 0, st
    for k in range(len(layers_a)):
        c0, c1 = srv.outputs(ids[4], k, na)
        assert (host(c0) == alone[k][0]).all() and (host(c1) == alone[k][1]).all(), f"layer {k} differs in the mix"
    # and the served outputs are the oracle's (sampled), for both networks
    for k, (s, f) in enumerate(zip(specs_a, filt_a)):
        P = layout.plan(N, s.c_i, s.c_o, s.h, s.w, s.f_w, s.stride)
        check_layer_points(P, ctx.primes, T, xa[k], f, ma[k], alone[k][0], alone[k][1], g, npts=24)
    idx_b = next(i for i, p in enumerate(plan) if p[1] == nb)
    net, x_b, m_b = others[0]
    for k, (s, f) in enumerate(zip(specs_b, filt_b)):
        P = layout.plan(N, s.c_i, s.c_o, s.h, s.w, s.f_w, s.stride)
        c0, c1 = srv.outputs(ids[idx_b], k, nb)
        check_layer_points(P, ctx.primes, T, host(x_b[k]), f, host(m_b[k]), host(c0), host(c1), g, npts=24)
    for i in ids.values():
        srv.release(i)
    assert srv.stats()["arena_used"] == 0
    srv.close()
    torch.cuda.synchronize()


def test_admission_waits_for_arena_space(setup):
    hconv, ctx, nets, g = setup
    specs_a, _, layers_a = nets["a"]
    probe = hconv.Server(ctx, arena_bytes=1 << 30, max_batch=4, streams=1)
    na = probe.add_net(layers_a)
    need = probe.request_bytes(na)
    probe.close()
    srv = hconv.Server(ctx, arena_bytes=2 * need + 4096, max_batch=4, streams=1)
    na = srv.add_net(layers_a)
    x, m = _inputs(ctx, specs_a, layers_a, g)
    dx, dm = [dev(v) for v in x], [dev(v) for v in m]
    ids = [srv.submit(na, dx, dm) for _ in range(5)]
    srv.step()
    st = srv.stats()
    assert st["admitted"] == 2 and st["queued"] == 3 and st["arena_used"] == 2 * need, st
    with pytest.raises(hconv.HcError) as e:
        srv.release(ids[0])  # still running
    assert e.value.status == -5
    done = []
    for _ in range(100000):
        srv.step()
        for i in srv.poll():
            done.append(i)
            srv.release(i)  # frees space for the queued ones
        if len(done) == 5:
            break
    assert sorted(done) == sorted(ids)
    st = srv.stats()
    assert st["completed"] == 5 and st["queued"] == 0 and st["arena_used"] == 0, st
    # identical inputs give identical outputs whatever the admission order
    srv.close()


def test_server_rejects_bad_configs(setup):
    hconv, ctx, nets, g = setup
    with pytest.raises(hconv.HcError):
        hconv.Server(ctx, arena_bytes=1 << 20, max_batch=17)
    with pytest.raises(hconv.HcError):
        hconv.Server(ctx, arena_bytes=1 << 20, max_batch=4, streams=0)
    srv = hconv.Server(ctx, arena_bytes=1 << 20, max_batch=4)
    with pytest.raises(hconv.HcError):  # one request cannot fit
        srv.add_net(nets["a"][2])
    srv.close()
