"""Seeded synthetic inputs for VaultX plots (keys, k mixes, request arrivals).

This module is shared by the oracle, the tests, the benchmark and the HIP-path
binding.  It holds none of the plotting method's arithmetic: no hashing, no
bucketing, no matching.  It only turns seeds into plot keys, k values and
arrival times.

Generator: SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), 64-bit state, golden-gamma
increment, the published two-multiply finaliser.

Recipes:
  * plot key from seed s: four consecutive outputs of SplitMix64(s), each
    written little-endian, concatenated -> 32 bytes (the 256-bit plot key the
    paper's plotter takes, section III-B).
  * batched mix (seed 4 by default): per plot one output x picks
    k = k_lo + x mod (k_hi - k_lo + 1), then four outputs form its key.
  * serving arrivals (seed 5 by default): per request one output picks k as
    above, four form the key, one more gives u = top 53 bits / 2**53 and the
    inter-arrival gap -ln(1 - u) / rate.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List

__all__ = [
    "SplitMix64", "derive_key", "batched_plan", "serving_arrivals",
    "PlotSpec", "Arrival", "SEED_SINGLE", "SEED_BATCHED", "SEED_SERVING",
    "SEED_SAMPLED_BUCKETS", "sampled_buckets",
]

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15

SEED_SINGLE = 0
SEED_BATCHED = 4
SEED_SERVING = 5
SEED_SAMPLED_BUCKETS = 31


class SplitMix64:
    """SplitMix64 stream; next() returns a Python int in [0, 2**64)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + GOLDEN_GAMMA) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def key(self) -> bytes:
        return b"".join(self.next().to_bytes(8, "little") for _ in range(4))

    def unit(self) -> float:
        """Uniform double in [0, 1) from the top 53 bits of one output."""
        return (self.next() >> 11) / float(1 << 53)


def derive_key(seed: int) -> bytes:
    """32-byte plot key: four SplitMix64(seed) outputs, little-endian."""
    return SplitMix64(seed).key()


@dataclass(frozen=True)
class PlotSpec:
    k: int
    key: bytes


def batched_plan(n_plots: int = 32, seed: int = SEED_BATCHED,
                 k_lo: int = 22, k_hi: int = 29) -> List[PlotSpec]:
    """n_plots plots with k uniform in [k_lo, k_hi] and independent keys."""
    g = SplitMix64(seed)
    span = k_hi - k_lo + 1
    out = []
    for _ in range(n_plots):
        k = k_lo + g.next() % span
        out.append(PlotSpec(k=k, key=g.key()))
    return out


@dataclass(frozen=True)
class Arrival:
    t: float          # arrival time in seconds from the start of the run
    k: int
    key: bytes


def serving_arrivals(n: int, rate_per_s: float, seed: int = SEED_SERVING,
                     k_lo: int = 22, k_hi: int = 30) -> List[Arrival]:
    """Poisson arrivals at rate_per_s, k uniform in [k_lo, k_hi]."""
    if rate_per_s <= 0:
        raise ValueError("rate_per_s must be positive")
    g = SplitMix64(seed)
    span = k_hi - k_lo + 1
    t = 0.0
    out = []
    for _ in range(n):
        k = k_lo + g.next() % span
        key = g.key()
        u = g.unit()
        t += -math.log1p(-u) / rate_per_s
        out.append(Arrival(t=t, k=k, key=key))
    return out


def sampled_buckets(n: int, seed: int = SEED_SAMPLED_BUCKETS,
                    bucket_bits: int = 24) -> List[int]:
    """n distinct bucket ids drawn with SplitMix64(seed), plus the first and
    last bucket; returned sorted."""
    g = SplitMix64(seed)
    nb = 1 << bucket_bits
    s = {0, nb - 1}
    while len(s) < n + 2:
        s.add(g.next() % nb)
    return sorted(s)
