"""Seeded synthetic inputs for DDM matching, shaped like the paper's workloads.

This module only draws coordinates. It performs none of the matching
arithmetic and is shared by the GPU path's tests and benchmarks and by the
CPU oracle's tests, so that both sides see byte-identical inputs.

Workload model (Sec. V, "Experimental Evaluation"): N extents split into
n subscriptions and m updates, placed uniformly in a routing space of side
L = 1e6, all with a common side chosen from the overlapping degree
alpha = N * l / L.  For d dimensions the same definition with volumes gives
side = L * (alpha / N) ** (1 / d).

Conventions shared by every generator here:
  * numpy ``default_rng`` (PCG64); coordinates drawn in float64 and rounded
    once to float32 (round to nearest even);
  * updates are drawn first, then subscriptions;
  * arrays are dimension-major float32 ``lo[d, count]``, ``hi[d, count]``;
  * for common-side boxes ``hi = f32(f32(lo) + f32(side))`` in float32;
  * ids are the implicit 0-based array index.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

L_SPACE = 1.0e6


@dataclasses.dataclass
class Instance:
    """One DDM problem: subscriptions S and updates U (dimension-major f32)."""
    s_lo: np.ndarray
    s_hi: np.ndarray
    u_lo: np.ndarray
    u_hi: np.ndarray
    name: str = ""
    side: float | None = None

    @property
    def d(self) -> int:
        return int(self.s_lo.shape[0])

    @property
    def n(self) -> int:
        return int(self.s_lo.shape[1])

    @property
    def m(self) -> int:
        return int(self.u_lo.shape[1])


def side_for_alpha(alpha: float, N: int, d: int, L: float = L_SPACE) -> float:
    """Common side that gives overlapping degree alpha for N boxes in L^d."""
    return float(L * (alpha / N) ** (1.0 / d))


def uniform_boxes(rng: np.random.Generator, count: int, d: int, side: float,
                  L: float = L_SPACE):
    """Lower corners uniform in [0, L)^d, common side; float32 outputs."""
    lo = rng.uniform(0.0, L, size=(d, count)).astype(np.float32)
    hi = (lo + np.float32(side)).astype(np.float32)
    return np.ascontiguousarray(lo), np.ascontiguousarray(hi)


def uniform_instance(seed, n: int, m: int, d: int, side: float,
                     name: str = "") -> Instance:
    rng = np.random.default_rng(seed)
    u_lo, u_hi = uniform_boxes(rng, m, d, side)
    s_lo, s_hi = uniform_boxes(rng, n, d, side)
    return Instance(s_lo, s_hi, u_lo, u_hi, name=name, side=side)


def split_regions(N: int) -> tuple[int, int]:
    """n subscriptions and m updates from N regions: n = floor(N/2), m = N - n."""
    n = N // 2
    return n, N - n


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def small_1d(seed: int = 0) -> Instance:
    """d=1, 5,000 + 5,000 segments, length 100 (alpha = 1), seed 0."""
    return uniform_instance(seed, 5000, 5000, 1, 100.0, name="d1_N1e4_alpha1")


def uniform_2d_1m(seed: int = 1) -> Instance:
    """d=2, 500,000 + 500,000 squares, side 1e6*sqrt(1/1e6) = 1,000 (alpha=1)."""
    side = side_for_alpha(1.0, 1_000_000, 2)
    return uniform_instance(seed, 500_000, 500_000, 2, side,
                            name="d2_N1e6_alpha1")


def hotspot_2d(seed: int = 2, n: int = 500_000, m: int = 500_000,
               n_hot: int = 16, sigma: float = 2.0e4, alpha: float = 100.0,
               sigma_log: float = 0.5) -> Instance:
    """d=2 regions clustered around 16 Gaussian hotspots, log-normal sides.

    Hotspot centres are uniform in [0, L)^2 with equal weights; a region's
    centre is its hotspot plus N(0, sigma^2) per axis (no clipping); its square
    side is s0 * exp(sigma_log * Z) with median s0 = L * sqrt(alpha / 1e6);
    the box is [c - s/2, c + s/2], each bound rounded once to float32.
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, L_SPACE, size=(n_hot, 2))
    s0 = L_SPACE * math.sqrt(alpha / 1.0e6)

    def draw(count):
        which = rng.integers(0, n_hot, size=count)
        c = centres[which].T + rng.normal(0.0, sigma, size=(2, count))
        s = s0 * np.exp(sigma_log * rng.standard_normal(count))
        lo = (c - s / 2.0).astype(np.float32)
        hi = (c + s / 2.0).astype(np.float32)
        return np.ascontiguousarray(lo), np.ascontiguousarray(hi)

    u_lo, u_hi = draw(m)
    s_lo, s_hi = draw(n)
    return Instance(s_lo, s_hi, u_lo, u_hi, name="d2_N1e6_hotspots_alpha100")


@dataclasses.dataclass
class BatchSpec:
    N: int
    d: int
    alpha: float
    seed: tuple


def batch_specs(seed: int = 3, count: int = 256, n_lo: float = 1e3,
                n_hi: float = 2e5, a_lo: float = 0.01, a_hi: float = 100.0):
    """Per-instance parameters of the batched workload (256 instances).

    N = 2*floor(logU[n_lo, n_hi] / 2) (split evenly), d ~ U{1,2,3},
    alpha ~ logU[a_lo, a_hi]; instance i's coordinates come from seed (seed, i).
    """
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        N = 2 * int(math.floor(math.exp(rng.uniform(math.log(n_lo),
                                                    math.log(n_hi))) / 2))
        d = int(rng.integers(1, 4))
        alpha = float(math.exp(rng.uniform(math.log(a_lo), math.log(a_hi))))
        specs.append(BatchSpec(N=N, d=d, alpha=alpha, seed=(seed, i)))
    return specs


def instance_from_spec(spec: BatchSpec) -> Instance:
    n, m = split_regions(spec.N)
    side = side_for_alpha(spec.alpha, spec.N, spec.d)
    return uniform_instance(list(spec.seed), n, m, spec.d, side,
                            name=f"N{spec.N}_d{spec.d}_a{spec.alpha:.3g}")


def batch_instances(seed: int = 3, count: int = 256) -> list[Instance]:
    return [instance_from_spec(s) for s in batch_specs(seed, count)]


@dataclasses.dataclass
class Request:
    arrival_s: float
    spec: BatchSpec


def serving_schedule(seed: int = 4, rate: float = 2000.0, duration_s: float = 60.0,
                     n_lo: float = 1e3, n_hi: float = 1e6, d: int = 3,
                     a_lo: float = 0.01, a_hi: float = 100.0) -> list[Request]:
    """Open-loop Poisson arrivals of match requests (d=3, log-uniform N, alpha).

    The whole schedule (arrival times and per-request seeds) is drawn from
    ``seed`` up front; request k's coordinates come from seed (seed, k).
    """
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    k = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration_s:
            break
        N = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        alpha = float(math.exp(rng.uniform(math.log(a_lo), math.log(a_hi))))
        reqs.append(Request(arrival_s=t, spec=BatchSpec(N=N, d=d, alpha=alpha,
                                                        seed=(seed, k))))
        k += 1
    return reqs


def tiny_adversarial(seed: int, n: int, m: int, d: int, grid: int = 8) -> Instance:
    """Small inputs on a coarse integer grid: many exact ties, touching ends,
    points (lo == hi), duplicates and nested intervals, plus signed zeros."""
    rng = np.random.default_rng(seed)

    def draw(count):
        a = rng.integers(-2, grid, size=(d, count)).astype(np.float64)
        b = a + rng.integers(0, 3, size=(d, count))
        lo = a.astype(np.float32)
        hi = b.astype(np.float32)
        z = rng.random((d, count)) < 0.1
        lo[z & (lo == 0)] = np.float32(-0.0)
        hi[(rng.random((d, count)) < 0.1) & (hi == 0)] = np.float32(-0.0)
        return np.ascontiguousarray(lo), np.ascontiguousarray(hi)

    u_lo, u_hi = draw(m)
    s_lo, s_hi = draw(n)
    return Instance(s_lo, s_hi, u_lo, u_hi, name=f"adv{seed}")


def random_lengths(seed: int, n: int, m: int, d: int, L: float = 1000.0,
                   max_len: float = 50.0) -> Instance:
    """Uniform lower ends, lengths uniform in [0, max_len) (variable lengths)."""
    rng = np.random.default_rng(seed)

    def draw(count):
        lo = rng.uniform(0.0, L, size=(d, count)).astype(np.float32)
        ln = rng.uniform(0.0, max_len, size=(d, count)).astype(np.float32)
        hi = (lo + ln).astype(np.float32)
        return np.ascontiguousarray(lo), np.ascontiguousarray(hi)

    u_lo, u_hi = draw(m)
    s_lo, s_hi = draw(n)
    return Instance(s_lo, s_hi, u_lo, u_hi, name=f"varlen{seed}")


def request_seed(seed) -> int:
    """64-bit seed of a request's device generator from its (seed, index)."""
    a, b = seed
    return (int(a) << 32) | int(b)


def device_instance(spec: BatchSpec, device: str = "cuda"):
    """A serving request's coordinates generated directly in device memory.

    Same recipe as uniform_instance (lower corners uniform on [0, L)^d drawn
    in float64 and rounded once to float32, hi = f32(lo + f32(side)), updates
    first), drawn from a torch device generator seeded with
    request_seed(spec.seed), so that arrivals need no host generation or
    upload.  Returns (s_lo, s_hi, u_lo, u_hi) float32 tensors [d, n] / [d, m].
    """
    import torch
    n, m = split_regions(spec.N)
    d = spec.d
    side = np.float32(side_for_alpha(spec.alpha, spec.N, d))
    g = torch.Generator(device=device)
    g.manual_seed(request_seed(spec.seed))
    lo = (torch.rand((d, m + n), dtype=torch.float64, device=device, generator=g)
          * L_SPACE).to(torch.float32)
    hi = lo + torch.tensor(side, dtype=torch.float32, device=device)
    return (lo[:, m:].contiguous(), hi[:, m:].contiguous(), lo[:, :m].contiguous(),
            hi[:, :m].contiguous())
