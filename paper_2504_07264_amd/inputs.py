"""Seeded synthetic inputs for the split-format DFT workloads.

This module only draws random numbers; it holds none of the transform's
arithmetic, so both the GPU path's tests and the oracle can be fed from it.

Recipe: a CPU ``torch.Generator`` seeded per workload; planes are drawn in the
order xr, xi, then any further planes (weights, upstream gradients), each of
shape ``[batch, n]`` in FP32.  ``uniform`` is ``2*rand - 1`` (uniform on
[-1, 1]); ``normal`` is ``randn`` (N(0, 1)).
"""
from __future__ import annotations

from dataclasses import dataclass

import torch


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    batch: int
    dist: str  # "uniform" or "normal"
    seed: int
    planes: int = 2  # number of [batch, n] planes drawn (xr, xi, wr, wi, ...)


# The workloads the transform is exercised on.  Sizes and distributions follow
# the batched-transform configurations the path is specified for.
SMALL_N16 = Workload("split_dft_n16_b256_uniform", 16, 256, "uniform", 0)
HEADLINE_N1024 = Workload("split_fft_n1024_b16384_normal", 1024, 16384, "normal", 1)
GRAD_N4096 = Workload("split_fft_grad_n4096_b4096_normal", 4096, 4096, "normal", 2, planes=4)
GRAD_FD_N64 = Workload("split_fft_grad_fd_n64_b8_normal", 64, 8, "normal", 2, planes=4)
PREC_N256 = Workload("split_fft_n256_b65536_uniform", 256, 65536, "uniform", 3)


def draw_planes(n: int, batch: int, dist: str, seed: int, planes: int = 2):
    """Draw ``planes`` FP32 tensors of shape [batch, n] from one seeded generator."""
    g = torch.Generator().manual_seed(seed)
    out = []
    for _ in range(planes):
        if dist == "uniform":
            t = torch.rand((batch, n), generator=g, dtype=torch.float32) * 2.0 - 1.0
        elif dist == "normal":
            t = torch.randn((batch, n), generator=g, dtype=torch.float32)
        else:
            raise ValueError("unknown distribution %r" % dist)
        out.append(t)
    return out


def draw(w: Workload):
    return draw_planes(w.n, w.batch, w.dist, w.seed, w.planes)


def ragged_lengths(count: int = 20000, kmin: int = 4, kmax: int = 16, seed: int = 4):
    """Lengths 2^k with k uniform on the integers [kmin, kmax], drawn first
    from the generator of ``seed``; returns (generator, lengths tensor)."""
    g = torch.Generator().manual_seed(seed)
    k = torch.randint(kmin, kmax + 1, (count,), generator=g)
    return g, torch.pow(2, k).to(torch.int64)


def draw_ragged(count: int = 20000, kmin: int = 4, kmax: int = 16, seed: int = 4, dist: str = "normal",
                planes: int = 4):
    """A ragged batch: lengths 2^k (k uniform on [kmin, kmax], drawn first),
    then ``planes`` flat FP32 planes of sum(lengths) values each, drawn in
    order from the same generator."""
    g, lengths = ragged_lengths(count, kmin, kmax, seed)
    total = int(lengths.sum())
    out = []
    for _ in range(planes):
        if dist == "normal":
            out.append(torch.randn(total, generator=g, dtype=torch.float32))
        else:
            out.append(torch.rand(total, generator=g, dtype=torch.float32) * 2.0 - 1.0)
    return lengths, out


# 20000 transforms of lengths 2^4 .. 2^16 (about 2^27.6 points), forward and
# adjoint in one grouped launch
RAGGED_COUNT, RAGGED_KMIN, RAGGED_KMAX, RAGGED_SEED = 20000, 4, 16, 4
