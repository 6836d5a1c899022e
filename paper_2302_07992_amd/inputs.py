"""Seeded synthetic workloads (grey images, payloads, keys).

This module only draws inputs; it holds none of the method's arithmetic, so
both the HIP path and the CPU oracle consume its bytes.  The recipe stands in
for the paper's 512x512 8-bit grey test corpus (classic test images and the
BOWS-2 set, Sec. IV), which is not available here:

    f(y, x) = 128 + sum_k a_k sin(2 pi (u_k x / N + v_k y / M) + phi_k) + sigma * n(y, x)
    image   = clip(rint(f), 0, 255) as uint8

with u_k, v_k ~ U(-4, 4) cycles per image, phi_k ~ U(0, 2 pi),
a_k ~ U(0.2, 1) rescaled to sum to 100, and n ~ N(0, 1).  The sinusoid
parameters come from numpy's PCG64(seed); the noise from a torch generator
seeded with the same seed on the device that draws the image.  Images drawn on
different devices can differ in a few pixels (float rounding), so a test always
hands the oracle the very bytes the GPU consumed.
"""
from __future__ import annotations

import math
from typing import Iterable, Sequence

import numpy as np
import torch

SIGMA_CYCLE = (1.0, 3.0, 8.0, 20.0)


def batch_sigma(i: int) -> float:
    """Noise sigma of image i in the 10,000-image batch workload."""
    return SIGMA_CYCLE[i % 4]


def batch_nsin(i: int) -> int:
    """Sinusoid count of image i in the batch workload (2..32)."""
    return 2 + (i * 7919) % 31


def key_pair(seed: int) -> tuple[int, int]:
    """(K1, K2) of the image with this seed."""
    return 2 * seed + 1, 2 * seed + 2


def _sin_params(seed: int, nsin: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(-4.0, 4.0, nsin)
    v = rng.uniform(-4.0, 4.0, nsin)
    phi = rng.uniform(0.0, 2.0 * math.pi, nsin)
    a = rng.uniform(0.2, 1.0, nsin)
    a = a * (100.0 / a.sum())
    return u, v, phi, a


def _field(seed: int, M: int, N: int, nsin: int, device) -> torch.Tensor:
    """Noise-free sinusoid field (float32, M x N), separable evaluation."""
    u, v, phi, a = _sin_params(seed, nsin)
    x = torch.arange(N, dtype=torch.float64) / N
    y = torch.arange(M, dtype=torch.float64) / M
    ax = 2 * math.pi * torch.from_numpy(u)[:, None] * x[None, :] + torch.from_numpy(phi)[:, None]  # K x N
    by = 2 * math.pi * torch.from_numpy(v)[:, None] * y[None, :]                                  # K x M
    amp = torch.from_numpy(a)[:, None]
    left = torch.cat([amp * torch.cos(by), amp * torch.sin(by)], 0).T.to(torch.float32)           # M x 2K
    right = torch.cat([torch.sin(ax), torch.cos(ax)], 0).to(torch.float32)                        # 2K x N
    return left.to(device) @ right.to(device)


def make_image(seed: int, M: int = 512, N: int = 512, nsin: int = 8, sigma: float = 3.0,
               device="cpu") -> torch.Tensor:
    """One M x N uint8 image on `device`."""
    f = _field(seed, M, N, nsin, device)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f = f + 128.0 + float(sigma) * torch.randn(M, N, generator=g, device=device, dtype=torch.float32)
    return torch.clamp(torch.round(f), 0, 255).to(torch.uint8)


def make_image_np(seed: int, M: int = 512, N: int = 512, nsin: int = 8, sigma: float = 3.0) -> np.ndarray:
    return make_image(seed, M, N, nsin, sigma, "cpu").numpy()


def fill_images(out: torch.Tensor, seeds: Sequence[int], nsins: Sequence[int], sigmas: Sequence[float]) -> None:
    """Fill out[i] (uint8, B x M x N, any device) with image(seeds[i])."""
    B, M, N = out.shape
    for i in range(B):
        out[i].copy_(make_image(int(seeds[i]), M, N, int(nsins[i]), float(sigmas[i]), out.device))


def make_band_image(seed: int, M: int, N: int, nsin: int = 8, sigma: float = 3.0, device="cpu",
                    band: int = 2048) -> torch.Tensor:
    """Large image drawn in row bands (keeps float temporaries small)."""
    u, v, phi, a = _sin_params(seed, nsin)
    out = torch.empty(M, N, dtype=torch.uint8, device=device)
    x = torch.arange(N, dtype=torch.float64) / N
    ax = 2 * math.pi * torch.from_numpy(u)[:, None] * x[None, :] + torch.from_numpy(phi)[:, None]
    right = torch.cat([torch.sin(ax), torch.cos(ax)], 0).to(torch.float32).to(device)
    amp = torch.from_numpy(a)[:, None]
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    for r0 in range(0, M, band):
        r1 = min(M, r0 + band)
        y = torch.arange(r0, r1, dtype=torch.float64) / M
        by = 2 * math.pi * torch.from_numpy(v)[:, None] * y[None, :]
        left = torch.cat([amp * torch.cos(by), amp * torch.sin(by)], 0).T.to(torch.float32).to(device)
        f = left @ right + 128.0 + float(sigma) * torch.randn(r1 - r0, N, generator=g, device=device)
        out[r0:r1] = torch.clamp(torch.round(f), 0, 255).to(torch.uint8)
    return out


def make_payload(seed: int, nbits: int, device="cpu") -> torch.Tensor:
    """Uniform random message of nbits bits, packed MSB-first (bytes)."""
    nbytes = (nbits + 7) // 8
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) + (1 << 32))
    msg = torch.randint(0, 256, (max(nbytes, 1),), generator=g, device=device, dtype=torch.int32).to(torch.uint8)
    if nbits % 8 and nbytes:
        msg[nbytes - 1] &= (0xFF << (8 - nbits % 8)) & 0xFF
    return msg[:nbytes]


def serving_sides(rng: np.random.Generator, n: int) -> np.ndarray:
    """Square image sides of the serving mix: 256..4096 weighted 30/40/15/10/5."""
    sides = np.array([256, 512, 1024, 2048, 4096])
    return rng.choice(sides, size=n, p=[0.30, 0.40, 0.15, 0.10, 0.05])


def seeds_range(n: int, first: int = 0) -> Iterable[int]:
    return range(first, first + n)
