"""Seeded synthetic inputs for the skyline workloads.

This module only draws random numbers and shapes them into point sets. It holds
none of the skyline method's arithmetic (no dominance test, no partitioning, no
scoring), so both the CPU oracle's tests and the GPU path's tests and benchmark
can take their inputs from here without sharing any of the method.

All arrays are float32 in SoA layout ``(d, N)``: ``pts[k, i]`` is coordinate k
of point i. Generators compute in float64 and round once to float32.

The paper's own generators are not specified (it only names uniform, correlated
and anticorrelated data, Section 5), so the recipes below are stand-ins with the
shapes of its workloads:

* ``uniform``: i.i.d. U[0,1).
* ``anticorrelated``: a plane offset eps ~ N(0, 0.05^2) per point and a uniform
  spread u ~ U[0,1)^d inside the plane, x = clip(0.5 + eps + (u - mean(u)), 0, 1),
  so sum(x) = d (0.5 + eps) before clipping.
* ``correlated``: v ~ U[0,1) per point, x_k = clip(v + N(0, 0.05^2), 0, 1).
* ``clustered``: 32 Gaussian clusters, centres U[0,1)^d, sigma 0.08, clipped.
* ``mixture_quantized``: 90% clustered and 10% anticorrelated points, clipped,
  then quantised to 1000 levels: k = min(floor(1000 x), 999), x = k / 1000.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform", "anticorrelated", "correlated", "clustered", "mixture_quantized",
    "discrete", "WORKLOADS", "workload", "batch_instances",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _f32(x: np.ndarray) -> np.ndarray:
    """(N, d) float64 -> contiguous (d, N) float32."""
    return np.ascontiguousarray(x.T.astype(np.float32))


def uniform(n: int, d: int, seed: int) -> np.ndarray:
    g = _rng(seed)
    return _f32(g.random((n, d)))


def anticorrelated(n: int, d: int, seed: int, sigma: float = 0.05) -> np.ndarray:
    g = _rng(seed)
    eps = g.normal(0.0, sigma, size=(n, 1))
    u = g.random((n, d))
    x = 0.5 + eps + (u - u.mean(axis=1, keepdims=True))
    return _f32(np.clip(x, 0.0, 1.0))


def correlated(n: int, d: int, seed: int, sigma: float = 0.05) -> np.ndarray:
    g = _rng(seed)
    v = g.random((n, 1))
    x = v + g.normal(0.0, sigma, size=(n, d))
    return _f32(np.clip(x, 0.0, 1.0))


def clustered(n: int, d: int, seed: int, k: int = 32, sigma: float = 0.08) -> np.ndarray:
    g = _rng(seed)
    centres = g.random((k, d))
    lab = g.integers(0, k, size=n)
    x = centres[lab] + g.normal(0.0, sigma, size=(n, d))
    return _f32(np.clip(x, 0.0, 1.0))


def mixture_quantized(n: int, d: int, seed: int, frac_ant: float = 0.10,
                      levels: int = 1000) -> np.ndarray:
    g = _rng(seed)
    n_ant = int(round(frac_ant * n))
    n_cl = n - n_ant
    sub = g.integers(0, 2**62, size=2)
    a = clustered(n_cl, d, int(sub[0])).T.astype(np.float64)
    b = anticorrelated(n_ant, d, int(sub[1])).T.astype(np.float64)
    x = np.concatenate([a, b], axis=0)
    x = x[g.permutation(n)]
    k = np.minimum(np.floor(x * levels), levels - 1)
    return _f32(k / levels)


def discrete(n: int, d: int, seed: int, levels: int) -> np.ndarray:
    """Values drawn from {0, 1/levels, ..., (levels-1)/levels}: forces ties and duplicates."""
    g = _rng(seed)
    return _f32(g.integers(0, levels, size=(n, d)) / float(levels))


# Named workloads: (generator, N, d, seed) plus the method options they are run with.
WORKLOADS = {
    "grid_uniform_10k_d4": dict(gen="uniform", n=10_000, d=4, seed=1,
                                opts=dict(partitioning="grid", p=16, m_per_dim=[2, 2, 2, 2], reps="none",
                                          grid_filter=True, merge="noseq")),
    "sliced_ant_1m_d6": dict(gen="anticorrelated", n=1_000_000, d=6, seed=2,
                             opts=dict(partitioning="sliced", p=16, reps="sorted",
                                       n_reps=64, merge="noseq")),
    "learned_ant_1m_d6": dict(gen="anticorrelated", n=1_000_000, d=6, seed=48,
                              opts=dict(partitioning="sliced", p=16, reps="learned",
                                        presort="learned", n_reps=64, merge="noseq")),
    "learned_clustered_1m_d6": dict(gen="clustered", n=1_000_000, d=6, seed=49,
                                    opts=dict(partitioning="sliced", p=16, reps="learned",
                                              presort="learned", n_reps=64, merge="noseq")),
    "angular_mix_10m_d8": dict(gen="mixture_quantized", n=10_000_000, d=8, seed=5,
                               opts=dict(partitioning="angular", p=64,
                                         m_per_dim=[2, 2, 2, 2, 2, 2, 1],
                                         grid_filter=True, grid_filter_m=4,
                                         reps="learned", n_reps=64,
                                         merge="global")),
}

# Training sets for the learned scorer: two anticorrelated and two clustered, 1M x 6.
TRAIN_SETS = [("anticorrelated", 40), ("anticorrelated", 41), ("clustered", 42), ("clustered", 43)]

_GEN = {"uniform": uniform, "anticorrelated": anticorrelated, "correlated": correlated,
        "clustered": clustered, "mixture_quantized": mixture_quantized}


def workload(name: str, n: int | None = None, seed: int | None = None) -> np.ndarray:
    """Points of a named workload; ``n`` and ``seed`` may be overridden for smaller cases."""
    w = WORKLOADS[name]
    return _GEN[w["gen"]](w["n"] if n is None else n, w["d"], w["seed"] if seed is None else seed)


def generate(gen: str, n: int, d: int, seed: int) -> np.ndarray:
    return _GEN[gen](n, d, seed)


def batch_instances(n_inst: int = 512, seed: int = 3, n_lo: int = 1_000, n_hi: int = 200_000):
    """Many independent instances: N_i log-uniform in [n_lo, n_hi], d_i uniform in {3..8},
    distribution uniform / correlated / anticorrelated at random. Returns a list of (d_i, N_i) arrays."""
    g = _rng(seed)
    out = []
    kinds = ["uniform", "correlated", "anticorrelated"]
    for i in range(n_inst):
        n_i = int(np.floor(np.exp(g.uniform(np.log(n_lo), np.log(n_hi)))))
        d_i = int(g.integers(3, 9))
        kind = kinds[int(g.integers(0, 3))]
        out.append(_GEN[kind](n_i, d_i, int(g.integers(0, 2**62))))
    return out
