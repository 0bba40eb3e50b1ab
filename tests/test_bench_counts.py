"""The benchmark's algorithmic work and byte counts (host only): bench.py's
per-layer counts, taken on the library's layout planner, against the counting
rules written out independently on the oracle's planner, and the ResNet-50
per-image totals against their closed values."""
import math
import types

import pytest

import bench
from oracle import layout as olayout
from paper_2401_16732_amd import hconv
from paper_2401_16732_amd import workloads as W


def _counts_library(spec, N, L, B, c0_mac=False):
    lay = hconv.plan_ring(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
    ly = types.SimpleNamespace(layout=lay, shape=(spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride))
    return bench.layer_counts(ly, B, N, L, c0_mac=c0_mac)


def _counts_rules(spec, N, L, B):
    """Counting rules: MAC = B O (G / T) 2 L N; butterflies = B (G + O) 2 L (N / 2) log2 N;
    mask adds = B c_out ho wo L; path bytes = B (G 2 L N + O L N + c_out L ho wo + c_out ho wo) 4."""
    P = olayout.plan(N, spec.c_i, spec.c_o, spec.h, spec.w, spec.f_w, spec.stride)
    bfly = (N // 2) * int(math.log2(N))
    return {
        "mac": B * P.O * (P.G // P.T) * 2 * L * N,
        "bfly_fwd": B * P.G * 2 * L * bfly,
        "bfly_inv": B * P.O * 2 * L * bfly,
        "mask": B * spec.c_o * P.ho * P.wo * L,
        "bytes_path": B * (P.G * 2 * L * N + P.O * L * N + spec.c_o * L * P.ho * P.wo + spec.c_o * P.ho * P.wo) * 4,
        "bytes_w": spec.c_o * P.G_w * L * N * 4,
    }


@pytest.mark.parametrize("net,N,L", [("resnet50_224", 8192, 3), ("resnet18_cifar", 8192, 3),
                                     ("resnet18_224", 16384, 4)])
def test_layer_counts_follow_the_counting_rules(net, N, L):
    for spec in W.NETS[net]():
        got = _counts_library(spec, N, L, B=16)
        exp = _counts_rules(spec, N, L, B=16)
        for k, v in exp.items():
            assert got[k] == v, (spec.name, k)


def test_resnet50_per_image_totals():
    """Per image at N = 8192, L = 3: 17.09 G MAC terms and 9.08 G butterflies
    (G + O summed over the 53 layers: 1,406 forward and 27,008 inverse
    transforms of 6 polynomials)."""
    tot = {}
    for spec in W.NETS["resnet50_224"]():
        for k, v in _counts_library(spec, 8192, 3, B=1).items():
            tot[k] = tot.get(k, 0) + v
    assert round(tot["mac"] / 1e9, 2) == 17.09
    assert round((tot["bfly_fwd"] + tot["bfly_inv"]) / 1e9, 2) == 9.08
    per_transform = (8192 // 2) * 13 * 6
    assert tot["bfly_fwd"] == 1406 * per_transform and tot["bfly_inv"] == 27008 * per_transform


def test_counts_with_c0_in_the_mac():
    """Where the MAC carries out c0's transform, the inverse NTT stage counts
    c1's butterflies only and the MAC stage c0's (half each); the totals and
    the interface bytes of the other stages are unchanged, and Yhat's c0 half
    leaves both the MAC's and the inverse NTT's bytes."""
    spec = W.ConvSpec(512, 2048, 7, 7, 1, 1)
    a = _counts_library(spec, 8192, 3, 16)
    b = _counts_library(spec, 8192, 3, 16, c0_mac=True)
    assert a["bfly_c0_mac"] == 0
    assert b["bfly_inv"] == b["bfly_c0_mac"] == a["bfly_inv"] // 2
    y_c0 = 16 * 2048 * 3 * 8192 * 4
    assert a["bytes_mac"] - b["bytes_mac"] == y_c0 and a["bytes_inv"] - b["bytes_inv"] == y_c0
    for k in ("mac", "bfly_fwd", "mask", "bytes_fwd", "bytes_path", "bytes_w"):
        assert a[k] == b[k], k
