"""Training recipe of the learned scorer (representatives and presort order).

Targets are the method's own dominance test in count mode (Def. 2): for every
training point t, dc(t) = #{s in S : t dominates s} against a fixed random
sample S of M points, computed on the GPU by ``sky_mlp_targets``. By default S
keeps only the sample points that the set's own Sorted representatives leave
undominated, so dc counts what the coordinate sum misses. The
scorer is fitted to y = -log1p(dc * N / M) / log1p(N): points that dominate much
of that residual get small scores, as the largest dominance regions are in
Region representatives (Section 4.1). The learned representatives mix the
smallest sums with the smallest learned scores, in the proportion that covers
the most of a sample. The weights
stay >= 0, so the scorer is a monotone scoring function and sorting by it is a
topological sort (Section 2).

Every step runs in the library's kernels; this module only moves tensors.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Scorer, mlp_targets, skyline


def targets(points: torch.Tensor, m: int = 65536, seed: int = 0, residual: bool = True,
            n_reps: int = 64) -> torch.Tensor:
    """Dominance-count targets for (d, N) device points against a seeded sample of m ids
    (``sky_mlp_targets``).

    With ``residual`` the sample points that the set's own Sorted representatives (the
    library's selection) dominate are left out, so the scorer learns where points dominate
    what the coordinate sum misses; its top scores then complement the sum's in the pool
    that learned representatives are picked from.
    """
    n = points.shape[1]
    m = min(m, n)
    rng = np.random.Generator(np.random.PCG64(seed))
    sample = torch.from_numpy(rng.choice(n, size=m, replace=False).astype(np.int32)).to(points.device)
    reps = None
    if residual:
        _, st = skyline(points, reps="sorted", n_reps=n_reps, return_stats=True)
        reps = torch.tensor(st.get("rep_ids", []), dtype=torch.int32, device=points.device)
    y, _ = mlp_targets(points, sample, reps)
    return y


def train_scorer(train_points: list[torch.Tensor], epochs: int = 3, batch: int = 4096, lr: float = 2e-3,
                 m: int = 65536, seed: int = 0, init: torch.Tensor | None = None,
                 residual: bool = True, balance: bool = False) -> tuple[Scorer, dict]:
    """Fit a scorer on the given (d, N) device point sets; returns (scorer, log)."""
    d = train_points[0].shape[0]
    sc = Scorer(d, init=init, seed=seed)
    sets = []
    for i, p in enumerate(train_points):
        y = targets(p, m, seed + i, residual)
        if balance:
            # every point with a non-zero target and as many zero-target points at
            # random, shuffled: the representatives come from the top of the
            # ranking, which the mostly-zero targets would otherwise drown out
            g = torch.Generator(device="cpu").manual_seed(seed + 1000 + i)
            pos = torch.nonzero(y < 0).flatten().cpu()
            zer = torch.nonzero(y >= 0).flatten().cpu()
            k = min(len(zer), max(len(pos), batch))
            pick = torch.cat([pos, zer[torch.randperm(len(zer), generator=g)[:k]]])
            pick = pick[torch.randperm(len(pick), generator=g)].to(p.device)
            sets.append((p[:, pick].contiguous(), y[pick].contiguous()))
        else:
            sets.append((p, y))
    log = {"epochs": epochs, "batch": batch, "lr": lr, "m": m, "balance": balance, "loss": [],
           "train_points": [int(q.shape[1]) for q, _ in sets]}
    for e in range(epochs):
        losses = [sc.train(q, y, epochs=1, batch=batch, lr=lr * (0.5 ** e)) for q, y in sets]
        log["loss"].append(float(np.mean(losses)))
    return sc, log
