"""Pins of the oracle's option variants: Region representatives, random
representatives and Random partitioning (Sections 3.1 and 4.1).

* SplitMix64 against its published output sequence (tests/golden).
* Region scores against the volume formula evaluated by hand, and the Region
  choice against float64 volumes on inputs without near ties.
* Random partitioning: equal sizes, the rank rule recomputed from an
  independent Python SplitMix64, and uniformity.
* Random representatives: distinct ids, uniform scores on the 2^-24 grid.
* The pipeline's result under every new option equals the brute-force skyline
  (Propositions 1 and 2: options never change the result).
"""
import os

import numpy as np
import pytest

import datagen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
M64 = 2**64 - 1


def _sm64_py(seed, i):
    """An independent Python SplitMix64 draw i (counter form)."""
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def test_splitmix64_published_sequence():
    want = [int(l) for l in open(os.path.join(HERE, "golden", "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    assert [oracle.splitmix64(1234567, i) for i in range(5)] == want
    assert [_sm64_py(1234567, i) for i in range(5)] == want


def test_region_scores_by_hand():
    x = np.array([[0.5, 0.0, 1.0, 0.25], [0.25, 0.0, 0.5, 0.75], [0.0, 0.0, 0.0, 0.5]], np.float32)
    # V = (1-x0)(1-x1)(1-x2): 0.5*0.75*1, 1*1*1, 0*0.5*1, 0.75*0.25*0.5
    assert oracle.region_scores(x).tolist() == [-0.375, -1.0, -0.0, -0.09375]
    with pytest.raises(ValueError):
        oracle.region_scores(np.array([[0.2, 1.5]], np.float32))
    with pytest.raises(ValueError):
        oracle.region_scores(np.array([[-0.1, 0.5]], np.float32))


def test_region_picks_largest_volumes():
    rng = np.random.default_rng(3)
    x = rng.random((4, 500)).astype(np.float32)
    v64 = np.prod(1.0 - x.astype(np.float64), axis=0)
    order = np.argsort(-v64, kind="stable")
    gaps = np.diff(-v64[order])
    assert gaps[:40].min() > 1e-6   # no near ties among the leaders
    assert oracle.select_reps(oracle.region_scores(x), 32).tolist() == order[:32].tolist()


@pytest.mark.parametrize("n,p", [(1000, 16), (997, 7), (5, 8), (1, 3), (64, 64)])
def test_random_cells_rule_and_sizes(n, p):
    seed = 12345
    cells = oracle.random_cells(n, p, seed)
    keys = [(_sm64_py(seed, i) >> 32, i) for i in range(n)]
    rank = {i: r for r, (_, i) in enumerate(sorted(keys))}
    assert cells.tolist() == [rank[i] * p // n for i in range(n)]
    sizes = np.bincount(cells, minlength=p)
    want = [-(-(j + 1) * n // p) - (-(-j * n // p)) for j in range(p)]   # ceil((j+1)n/p) - ceil(jn/p)
    assert sizes.tolist() == want


def test_random_cells_look_random():
    n, p = 20000, 16
    a, b = oracle.random_cells(n, p, 1), oracle.random_cells(n, p, 2)
    assert (a != b).mean() > 0.9   # another seed, another partition
    ids = np.arange(n)
    for j in range(p):   # every partition spans the id range evenly
        m = ids[a == j].mean()
        assert abs(m - n / 2) < 0.06 * n


def test_random_scores_grid_and_uniformity():
    s = oracle.random_scores(50000, 7)
    assert s.min() >= 0.0 and s.max() < 1.0
    assert np.all(s * 2**24 == np.floor(s * 2**24))
    assert abs(s.mean() - 0.5) < 0.01
    hist = np.bincount((s * 10).astype(int), minlength=10)
    chi2 = ((hist - 5000.0) ** 2 / 5000.0).sum()
    assert chi2 < 30   # 9 degrees of freedom
    assert not np.array_equal(s[:100], oracle.random_scores(100, 8))
    ids = oracle.select_reps(s, 64)
    assert len(set(ids.tolist())) == 64


@pytest.mark.parametrize("opts", [
    dict(partitioning="random", p=8, reps="none"),
    dict(partitioning="random", p=5, reps="sorted", n_reps=16, merge="global"),
    dict(partitioning="sliced", p=6, reps="region", n_reps=16),
    dict(partitioning="angular", p=4, m_per_dim=[2, 2], reps="random", n_reps=32),
    dict(partitioning="random", p=16, reps="region", n_reps=8, grid_filter=True, grid_filter_m=3),
])
def test_pipeline_variants_equal_brute_force(opts):
    for seed, x in enumerate([datagen.anticorrelated(3000, 3, 31), datagen.uniform(2000, 3, 32),
                              datagen.discrete(2500, 3, 33, 4)]):
        ids, st = oracle.pipeline(x, seed=seed + 11, threads=2, **opts)
        assert np.array_equal(ids, oracle.sky_brute(x))
        if opts["partitioning"] == "random":
            n, p = x.shape[1], opts["p"]
            assert st["part_sizes"].tolist() == [-(-(j + 1) * n // p) - (-(-j * n // p)) for j in range(p)]


def test_region_pipeline_needs_unit_range():
    x = datagen.anticorrelated(200, 3, 1) * 2.0
    with pytest.raises(ValueError):
        oracle.pipeline(x, partitioning="sliced", p=4, reps="region", n_reps=8)
