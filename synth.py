"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws numbers. It holds none of the rescaling arithmetic, so
both the FP64 CPU oracle side and the GPU side can take their inputs from it
without sharing any method code.

Every generator uses numpy's PCG64 (``numpy.random.default_rng(seed)``) and
returns float32 arrays in NCHW order. The image sets stand in for the 1024x1024
RGB face photographs the paper times on (Sec. 6, "Hardware & Datasets"); that
dataset is not used here.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "uniform", "normal", "smooth", "bf16_round", "f16_round",
    "Request", "request_stream",
]


def uniform(seed: int, shape) -> np.ndarray:
    """Values uniform in [0, 1), float32."""
    return np.random.default_rng(seed).random(shape, dtype=np.float32)


def normal(seed: int, shape, std: float = 1.0, mean: float = 0.0) -> np.ndarray:
    """Gaussian values, float32 (``std`` is the standard deviation)."""
    g = np.random.default_rng(seed).standard_normal(shape, dtype=np.float32)
    if std != 1.0:
        g *= np.float32(std)
    if mean != 0.0:
        g += np.float32(mean)
    return g


def smooth(seed: int, shape, sigma: float = 16.0) -> np.ndarray:
    """Smooth fields: white noise blurred by a separable Gaussian of ``sigma``
    pixels over the last two axes, then min-max scaled into [0, 1).

    These mimic natural images (strong low-frequency content) so that the
    interpolation is exercised on realistic, correlated data.
    """
    from scipy.ndimage import gaussian_filter1d

    g = np.random.default_rng(seed).standard_normal(shape, dtype=np.float32)
    g = gaussian_filter1d(g, sigma, axis=-1, mode="mirror")
    g = gaussian_filter1d(g, sigma, axis=-2, mode="mirror")
    lo, hi = float(g.min()), float(g.max())
    scale = (1.0 - 2.0 ** -20) / max(hi - lo, 1e-30)
    return ((g - lo) * scale).astype(np.float32)


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest even) and return
    them widened back to float32 (so they are exactly representable in both)."""
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(
        torch.bfloat16).to(torch.float32).numpy()


def f16_round(a: np.ndarray) -> np.ndarray:
    """Round float32 values to IEEE binary16 (RNE), widened back to float32."""
    return np.ascontiguousarray(a, dtype=np.float32).astype(np.float16).astype(np.float32)


@dataclass
class Request:
    """One rescale request of the serving workload."""
    idx: int
    arrive_s: float      # arrival time relative to the stream start
    p: int
    q: int
    method: int          # 0 nearest, 1 bilinear, 2 bicubic
    pad: int             # 0 zero, 1 replicate, 2 reflect
    dtype: int           # 0 fp32, 1 bf16
    c: int
    h: int
    w: int
    seed: int


def request_stream(seed: int, count: int, rate_per_s: float, c: int = 3,
                   hw_lo: int = 64, hw_hi: int = 2048, pq_max: int = 8):
    """A Poisson arrival stream of rescale requests.

    Sizes are uniform integers in [hw_lo, hw_hi], p and q uniform in
    1..pq_max, the method uniform over nearest/bilinear/bicubic and the
    storage type fp32 or bf16 with equal odds. Each request carries its own
    seed for its pixel values.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count) if rate_per_s > 0 else np.zeros(count)
    t = np.cumsum(gaps) - gaps[0]
    hs = rng.integers(hw_lo, hw_hi + 1, size=count)
    ws = rng.integers(hw_lo, hw_hi + 1, size=count)
    ps = rng.integers(1, pq_max + 1, size=count)
    qs = rng.integers(1, pq_max + 1, size=count)
    ms = rng.integers(0, 3, size=count)
    pads = rng.integers(0, 3, size=count)
    dts = rng.integers(0, 2, size=count)
    seeds = rng.integers(0, 2 ** 31 - 1, size=count)
    return [Request(i, float(t[i]), int(ps[i]), int(qs[i]), int(ms[i]), int(pads[i]),
                    int(dts[i]), c, int(hs[i]), int(ws[i]), int(seeds[i]))
            for i in range(count)]

