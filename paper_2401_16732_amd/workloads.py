"""Seeded synthetic workloads: ResNet-shaped conv-layer lists and input generators.

This module holds no homomorphic arithmetic. It only states layer shapes and
draws seeded random inputs, so that the CPU oracle and the GPU path are fed the
same values.

The paper evaluates on CIFAR-100 / TinyImageNet with trained ResNet and VGG
models (Experimental Results section). No dataset or trained weight is used
here: weights are uniform int8, activations are uniform integers in a stated
range, and ciphertext limbs are uniform residues (uniform mod q by CRT).
Draw order per workload: weights, then activations, then ciphertext limbs,
then masks.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np


@dataclass(frozen=True)
class ConvSpec:
    """One convolution layer: c_i -> c_o channels on an h x w input.

    f_w is the (odd) filter width and `stride` the stride; padding is 'same'
    ((f_w - 1) / 2), as in the paper's zero-padded inputs (Proposed
    Convolution with DRot section).
    """
    c_i: int
    c_o: int
    h: int
    w: int
    f_w: int
    stride: int = 1
    name: str = ""


def resnet18_cifar() -> List[ConvSpec]:
    """ResNet-18 conv layers on a 32x32x3 input (20 convolutions)."""
    L: List[ConvSpec] = [ConvSpec(3, 64, 32, 32, 3, 1, "stem")]
    L += [ConvSpec(64, 64, 32, 32, 3, 1, f"s1.{k}") for k in range(4)]
    size, cin = 32, 64
    for st, cout in enumerate((128, 256, 512), start=2):
        L.append(ConvSpec(cin, cout, size, size, 3, 2, f"s{st}.b1.c1"))
        half = size // 2
        L.append(ConvSpec(cout, cout, half, half, 3, 1, f"s{st}.b1.c2"))
        L.append(ConvSpec(cin, cout, size, size, 1, 2, f"s{st}.b1.proj"))
        L += [ConvSpec(cout, cout, half, half, 3, 1, f"s{st}.b2.c{k}") for k in (1, 2)]
        size, cin = half, cout
    return L


def resnet18_224() -> List[ConvSpec]:
    """ResNet-18 conv layers on a 224x224x3 input (7x7/2 stem; 20 convolutions)."""
    L: List[ConvSpec] = [ConvSpec(3, 64, 224, 224, 7, 2, "stem")]
    L += [ConvSpec(64, 64, 56, 56, 3, 1, f"s1.{k}") for k in range(4)]
    size, cin = 56, 64
    for st, cout in enumerate((128, 256, 512), start=2):
        L.append(ConvSpec(cin, cout, size, size, 3, 2, f"s{st}.b1.c1"))
        half = size // 2
        L.append(ConvSpec(cout, cout, half, half, 3, 1, f"s{st}.b1.c2"))
        L.append(ConvSpec(cin, cout, size, size, 1, 2, f"s{st}.b1.proj"))
        L += [ConvSpec(cout, cout, half, half, 3, 1, f"s{st}.b2.c{k}") for k in (1, 2)]
        size, cin = half, cout
    return L


def resnet50_224() -> List[ConvSpec]:
    """ResNet-50 conv layers on a 224x224x3 input (53 convolutions).

    Bottleneck blocks [3, 4, 6, 3] at 56/28/14/7 with the stride in the 3x3
    and 1x1 stride-2 projections.
    """
    L: List[ConvSpec] = [ConvSpec(3, 64, 224, 224, 7, 2, "stem")]
    cin, size = 64, 56
    for st, (width, nblk) in enumerate(((64, 3), (128, 4), (256, 6), (512, 3)), start=1):
        cout = width * 4
        for b in range(nblk):
            s = 2 if (b == 0 and st > 1) else 1
            L.append(ConvSpec(cin, width, size, size, 1, 1, f"s{st}.b{b}.c1"))
            L.append(ConvSpec(width, width, size, size, 3, s, f"s{st}.b{b}.c2"))
            osz = size // s
            L.append(ConvSpec(width, cout, osz, osz, 1, 1, f"s{st}.b{b}.c3"))
            if b == 0:
                L.append(ConvSpec(cin, cout, size, size, 1, s, f"s{st}.b{b}.proj"))
            cin, size = cout, osz
    return L


NETS = {"resnet18_cifar": resnet18_cifar, "resnet18_224": resnet18_224, "resnet50_224": resnet50_224}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gen_filters(g: np.random.Generator, spec: ConvSpec) -> np.ndarray:
    """int8 filters [c_o][c_i][f_w][f_w], uniform in [-128, 127]."""
    return g.integers(-128, 128, size=(spec.c_o, spec.c_i, spec.f_w, spec.f_w), dtype=np.int64).astype(np.int8)


def gen_activations(g: np.random.Generator, spec: ConvSpec, lo: int, hi: int, batch: int = 1) -> np.ndarray:
    """Integer activations [batch][c_i][h][w], uniform in [lo, hi)."""
    return g.integers(lo, hi, size=(batch, spec.c_i, spec.h, spec.w), dtype=np.int64)


def gen_ct_limbs(g: np.random.Generator, lead_shape: Sequence[int], primes: Sequence[int], n: int) -> np.ndarray:
    """Uniform residues shaped lead_shape + [L][n]; limb l is uniform in [0, primes[l])."""
    L = len(primes)
    out = np.empty(tuple(lead_shape) + (L, n), dtype=np.uint32)
    for l, q in enumerate(primes):
        out[..., l, :] = g.integers(0, q, size=tuple(lead_shape) + (n,), dtype=np.uint64).astype(np.uint32)
    return out


def gen_mask(g: np.random.Generator, shape: Sequence[int], t: int) -> np.ndarray:
    """Server masks r, uniform in [0, t), as uint32."""
    return g.integers(0, t, size=tuple(shape), dtype=np.uint64).astype(np.uint32)


def gen_ct_limbs_torch(gen, lead_shape, primes, n, device):
    """Same distribution as gen_ct_limbs, drawn on the device by torch's seeded
    generator (used where host generation of many GiB would dominate)."""
    import torch
    L = len(primes)
    out = torch.empty(tuple(lead_shape) + (L, n), dtype=torch.int32, device=device)
    for l, q in enumerate(primes):
        v = torch.randint(0, q, tuple(lead_shape) + (n,), generator=gen, device=device, dtype=torch.int64)
        out[..., l, :] = v.to(torch.int32)
    return out
