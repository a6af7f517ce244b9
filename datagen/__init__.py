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
* ``household_like`` and ``housing_like``: synthetic stand-ins with the sizes and
  the value structure of the paper's two real datasets (Section 5: a household's
  per-minute electricity readings, 2,049,280 x 7; housing records, 3,569,678 x 7).
  None of their values is used or reproduced; the generators only draw numbers
  with that kind of structure: a few latent factors shared by correlated
  attributes, heavy tails, readings on fixed steps (many exact ties),
  zero-inflated attributes; every attribute is scaled to [0, 1].
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform", "anticorrelated", "correlated", "clustered", "mixture_quantized",
    "discrete", "household_like", "housing_like", "WORKLOADS", "workload", "batch_instances",
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


def _unit_steps(x: np.ndarray, steps: int) -> np.ndarray:
    """Each column scaled to [0, 1] by its range, then put on `steps` equal steps."""
    lo = x.min(axis=0, keepdims=True)
    hi = x.max(axis=0, keepdims=True)
    u = (x - lo) / np.where(hi > lo, hi - lo, 1.0)
    return np.round(u * steps) / steps


def household_like(n: int, d: int, seed: int) -> np.ndarray:
    """Stand-in shaped like per-minute household power readings (d = 7 attributes):
    a lognormal load drives active power and current almost linearly, reactive power
    weakly, the voltage sags slightly with load, and three sub-meters read 0 most of
    the time; readings on 1/1000 steps of each attribute's range."""
    if d != 7:
        raise ValueError("household_like has 7 attributes")
    g = _rng(seed)
    load = g.lognormal(-0.5, 0.9, size=n)
    active = load * (1.0 + 0.02 * g.standard_normal(n))
    reactive = 0.1 * load ** 0.5 * g.gamma(2.0, 0.5, size=n)
    voltage = 240.0 - 1.5 * load + 3.0 * g.standard_normal(n)
    current = 4.2 * active + 0.2 * g.standard_normal(n)
    subs = []
    for rate, scale in ((0.08, 30.0), (0.12, 20.0), (0.35, 15.0)):
        on = g.random(n) < rate * (0.5 + np.minimum(load, 3.0) / 3.0)
        subs.append(np.where(on, np.floor(g.gamma(2.0, scale / 2.0, size=n)), 0.0))
    x = np.stack([active, reactive, voltage, current] + subs, axis=1)
    return _f32(_unit_steps(x, 1000))


def housing_like(n: int, d: int, seed: int) -> np.ndarray:
    """Stand-in shaped like housing records (d = 7 attributes): a lognormal size
    factor drives living area, rooms and price; the lot area is heavy tailed; the
    construction year is an integer; counts take integer or half-integer values.
    Smaller is better in every coordinate, so the size-like attributes and the
    year enter as 1 - value (cheap, large, recent houses form the skyline)."""
    if d != 7:
        raise ValueError("housing_like has 7 attributes")
    g = _rng(seed)
    size = g.lognormal(0.0, 0.45, size=n)
    area = np.round(1800.0 * size * np.exp(0.15 * g.standard_normal(n)) / 10.0) * 10.0
    beds = np.clip(np.round(3.0 * size + 0.7 * g.standard_normal(n)), 0, 12)
    baths = np.clip(np.round(2.0 * (2.0 * size + 0.5 * g.standard_normal(n))) / 2.0, 0.5, 10)
    price = np.round(3.0e5 * size ** 1.2 * np.exp(0.35 * g.standard_normal(n)), -3)
    lot = np.round(6000.0 * g.pareto(1.6, size=n) + 2000.0 * size, -1)
    year = np.round(np.clip(1975.0 + 25.0 * g.standard_normal(n) + 10.0 * (size - 1.0), 1850, 2022))
    tax = np.round(0.011 * price * np.exp(0.2 * g.standard_normal(n)))
    x = _unit_steps(np.stack([price, area, beds, baths, lot, year, tax], axis=1), 4096)
    x[:, 1:6] = 1.0 - x[:, 1:6]   # a buyer's preference: more area, rooms, lot and a newer house are better
    return _f32(x)


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

# Stand-ins shaped like the paper's two real datasets (sizes from its Section 5).
REAL_SHAPED = {"HOU-shaped": ("household_like", 2_049_280, 7, 71), "RES-shaped": ("housing_like", 3_569_678, 7, 72)}

# Training sets for the learned scorer: two anticorrelated and two clustered, 1M x 6.
TRAIN_SETS = [("anticorrelated", 40), ("anticorrelated", 41), ("clustered", 42), ("clustered", 43)]

_GEN = {"uniform": uniform, "anticorrelated": anticorrelated, "correlated": correlated,
        "clustered": clustered, "mixture_quantized": mixture_quantized,
        "household_like": household_like, "housing_like": housing_like}


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
