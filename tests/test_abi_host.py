"""The C-ABI library on the CPU: it loads, exports every declared entry point,
and its host-only logic (layout planner, ring parameters) agrees with the
oracle's independent implementation. No kernel is launched here."""
import ctypes
import os
import re

import pytest

from oracle import layout as olayout
from oracle import params as oparams
from paper_2401_16732_amd import hconv
from paper_2401_16732_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "hc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:hc_status|void|const char\s*\*)\s*(hc_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = hconv.load()
    names = declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(hconv.SYMBOLS)


def test_status_strings():
    lib = hconv.load()
    for s, text in [(0, b"ok"), (-1, b"invalid argument"), (-2, b"unsupported"), (-4, b"device error")]:
        assert lib.hc_status_string(s) == text


@pytest.mark.parametrize("N,L,t", [(4096, 2, 2 ** 17), (8192, 3, 2 ** 20), (16384, 4, 2 ** 24), (1024, 1, 3),
                                   (2048, 4, 2 ** 30)])
def test_ring_params_match_oracle(N, L, t):
    primes, deltas = hconv.ring_params(N, L, t)
    assert primes == oparams.rns_primes(N, L)
    assert deltas == oparams.delta_limbs(primes, t)


def _same_plan(N, spec):
    lay = hconv.plan_ring(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
    P = olayout.plan(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
    got = (lay.sub, lay.s, lay.h_enc, lay.w_enc, lay.pad, lay.h_pad, lay.w_pad, lay.footprint, lay.tiled, lay.cn,
           lay.tiles, lay.rows_out_per_tile, lay.in_cts, lay.w_cts, lay.out_cts, lay.ho, lay.wo)
    exp = (P.sub, P.s, P.he, P.we, P.pad, P.hp, P.wp, P.F, int(P.tiled), P.c_n, P.T, P.r_o, P.G, P.G_w, P.O,
           P.ho, P.wo)
    assert got == exp, (spec, got, exp)


@pytest.mark.parametrize("net,N", [("resnet18_cifar", 8192), ("resnet50_224", 8192), ("resnet18_224", 16384),
                                   ("resnet18_cifar", 1024), ("resnet50_224", 4096)])
def test_planner_matches_oracle_on_network_layers(net, N):
    for spec in W.NETS[net]():
        try:
            olayout.plan(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
        except ValueError:
            with pytest.raises(hconv.HcError):
                hconv.plan_ring(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
            continue
        _same_plan(N, spec)


def test_planner_matches_oracle_on_odd_shapes():
    g = W.rng(77)
    for _ in range(300):
        N = int(2 ** g.integers(10, 15))
        f = int(g.choice([1, 3, 5, 7]))
        spec = W.ConvSpec(int(g.integers(1, 40)), int(g.integers(1, 9)), int(g.integers(1, 150)),
                          int(g.integers(1, 150)), f, int(g.integers(1, 4)))
        try:
            olayout.plan(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
        except ValueError:
            with pytest.raises(hconv.HcError):
                hconv.plan_ring(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
            continue
        _same_plan(N, spec)


def test_planner_rejects_bad_shapes():
    with pytest.raises(hconv.HcError) as e:
        hconv.plan_ring(4096, 4, 4, 8, 8, 2, 1)
    assert e.value.status == -2
    with pytest.raises(hconv.HcError) as e:
        hconv.plan_ring(3000, 4, 4, 8, 8, 3, 1)
    assert e.value.status == -2
    with pytest.raises(hconv.HcError) as e:
        hconv.plan_ring(4096, 0, 4, 8, 8, 3, 1)
    assert e.value.status == -1


def test_client_and_protocol_entry_points_reject_null_handles():
    """Argument checks that return before any device call: a null context or
    layer is HC_EINVAL, with a message for hc_last_error."""
    lib = hconv.load()
    n = None
    sz = ctypes.c_size_t()
    assert lib.hc_encrypt_online(n, n, n, n, 1, n) == -1
    assert lib.hc_encrypt_zero(n, n, n, n, n, 1, n, 0, n) == -1
    assert lib.hc_decrypt(n, n, n, n, 1, n, 0, n) == -1
    assert lib.hc_decrypt_extracted(n, n, n, n, n, 1, n, 0, n) == -1
    assert lib.hc_decrypt_workspace_size(n, 1, ctypes.byref(sz)) == -1
    assert lib.hc_batch_encode(n, n, n, 1, n) == -1
    assert lib.hc_batch_decode(n, n, n, 1, n) == -1
    assert lib.hc_encrypt_plain(n, n, n, n, 1, n) == -1
    assert lib.hc_act_workspace_size(n, 1, ctypes.byref(sz)) == -1
    assert lib.hc_act_pmult(n, n, n, n, n, 1, n, 0, n) == -1
    assert lib.hc_act_combine(n, n, n, n, n, n, 1, n) == -1
    assert lib.hc_last_error() != b""


def test_new_entry_points_reject_null_handles():
    """The conventional convolution, rotation-order encoding, pipelined batch,
    no-allocation conv, per-batch-size tuning, MAC grid cap and VALU probe entry
    points refuse null handles and outputs before any device call."""
    lib = hconv.load()
    n = None
    sz = ctypes.c_size_t()
    assert lib.hc_cconv_create(n, n, n, 10, n, n) == -1
    assert lib.hc_cconv_info(n, n, n) == -1
    assert lib.hc_cconv_keys_size(n, ctypes.byref(sz)) == -1
    assert lib.hc_cconv_keygen_workspace_size(n, ctypes.byref(sz)) == -1
    assert lib.hc_cconv_keygen(n, n, n, n, n, n, 0, n) == -1
    assert lib.hc_cconv_workspace_size(n, 1, ctypes.byref(sz)) == -1
    assert lib.hc_cconv_run(n, n, n, n, 1, n, 0, n) == -1
    lib.hc_cconv_destroy(n)  # a no-op
    assert lib.hc_rot_encode(n, n, n, 1, n) == -1
    assert lib.hc_rot_decode(n, n, n, 1, n, 0, n) == -1
    assert lib.hc_batch_run_pipelined(n, n, n, n, n, 1 << 20, 3, n) == -1
    assert lib.hc_conv_masked_noalloc(n, n, n, n, n, 1, n) == -1
    t = hconv.Tuning()
    assert lib.hc_layer_get_tuning_for(n, 1, ctypes.byref(t)) == -1
    assert lib.hc_valu_probe(0, n) == -1
    cap = ctypes.c_uint32()
    assert lib.hc_batch_get_mac_cap(n, ctypes.byref(cap)) == -1
    assert lib.hc_batch_set_mac_cap(n, 0) == -1
    assert lib.hc_last_error() != b""
