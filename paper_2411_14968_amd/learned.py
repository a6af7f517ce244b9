"""Training recipe of the learned scorer (representatives and presort order).

Targets are the method's own dominance test in count mode (Def. 2): for every
training point t, dc(t) = #{s in S : t dominates s} against a fixed random
sample S of M points, computed on the GPU by ``sky_domcount``. The scorer is
fitted to y = -log1p(dc * N / M) / log1p(N), so points that dominate much of the
data get small scores and are chosen first, as the largest dominance regions
are in Region representatives (Section 4.1). Its weights stay >= 0, so it is a
monotone scoring function and sorting by it is a topological sort (Section 2).

Every step runs in the library's kernels; this module only moves tensors.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import Scorer, domcount


def targets(points: torch.Tensor, m: int = 65536, seed: int = 0) -> torch.Tensor:
    """Dominance-count targets for (d, N) device points against a seeded sample of m ids."""
    n = points.shape[1]
    m = min(m, n)
    rng = np.random.Generator(np.random.PCG64(seed))
    sample = torch.from_numpy(rng.choice(n, size=m, replace=False).astype(np.int32)).to(points.device)
    dc = domcount(points, sample).to(torch.float32)
    return -torch.log1p(dc * (n / m)) / math.log1p(n)


def train_scorer(train_points: list[torch.Tensor], epochs: int = 3, batch: int = 4096, lr: float = 2e-3,
                 m: int = 65536, seed: int = 0, init: torch.Tensor | None = None) -> tuple[Scorer, dict]:
    """Fit a scorer on the given (d, N) device point sets; returns (scorer, log)."""
    d = train_points[0].shape[0]
    sc = Scorer(d, init=init, seed=seed)
    ys = [targets(p, m, seed + i) for i, p in enumerate(train_points)]
    log = {"epochs": epochs, "batch": batch, "lr": lr, "m": m, "loss": []}
    for e in range(epochs):
        losses = [sc.train(p, y, epochs=1, batch=batch, lr=lr * (0.5 ** e)) for p, y in zip(train_points, ys)]
        log["loss"].append(float(np.mean(losses)))
    return sc, log
