"""GPU parity of the paper's option variants: Random partitioning (Section 3.1),
Region representatives, random representatives and Sorted representatives taken
per partition (Section 4.1).

Every case compares the library with the oracle on the same seeded input and
seed: the skyline ids, and every intermediate the two share (partition sizes
and survivors, local skyline sizes, representative ids and their self-filter,
counts after the filters, size of u). Both the captured-graph path (no stats)
and the eager path (stats) are checked. Expected values come from ``oracle``.
"""
import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu
THREADS = 4


@pytest.fixture(scope="module")
def sky():
    import paper_2411_14968_amd as m
    assert torch.cuda.is_available()
    return m


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _check(st, ost):
    for k in ("n_after_grid", "n_after_reps", "size_u", "size_sky"):
        assert st[k] == ost[k], k
    assert st["part_sizes"] == ost["part_sizes"].tolist()
    assert st["part_kept"] == ost["part_kept"].tolist()
    assert st["local_sizes"] == ost["local_sizes"].tolist()
    if "rep_ids" in ost:
        assert st["rep_ids"] == ost["rep_ids"].tolist()
        assert st["rep_keep"] == ost["rep_keep"].tolist()
        assert st["n_reps_kept"] == ost["n_reps_kept"]


OPTS = [dict(partitioning="random", p=16, reps="none"),
        dict(partitioning="random", p=5, reps="sorted", n_reps=32, merge="global"),
        dict(partitioning="random", p=1, reps="random", n_reps=16),
        dict(partitioning="sliced", p=16, reps="region", n_reps=64),
        dict(partitioning="grid", p=16, m_per_dim=[2, 2, 2, 2], reps="region", n_reps=16, presort="sum"),
        dict(partitioning="angular", p=8, m_per_dim=[2, 2, 2], reps="random", n_reps=64),
        dict(partitioning="random", p=64, reps="region", n_reps=8, grid_filter=True, grid_filter_m=3),
        dict(partitioning="sliced", p=16, reps="sorted_part", n_reps=64),
        dict(partitioning="sliced", p=7, reps="sorted_part", n_reps=20, merge="global", presort="sum"),
        dict(partitioning="sliced", p=100, reps="sorted_part", n_reps=64),
        dict(partitioning="grid", p=16, m_per_dim=[2, 2, 2, 2], reps="sorted_part", n_reps=64, grid_filter=True),
        dict(partitioning="angular", p=8, m_per_dim=[2, 2, 2], reps="sorted_part", n_reps=16),
        dict(partitioning="random", p=5, reps="sorted_part", n_reps=64),
        dict(partitioning="none", reps="sorted_part", n_reps=64)]


@pytest.mark.parametrize("opts", OPTS)
def test_variants_match_oracle(sky, orc, opts):
    xs = [datagen.anticorrelated(20_000, 4, 41), datagen.uniform(15_000, 4, 42), datagen.discrete(10_000, 4, 43, 5)]
    for seed, x in zip((0, 7, 2**63 + 5), xs):
        oids, ost = orc.pipeline(x, threads=THREADS, seed=seed, **opts)
        ids, st = sky.skyline(_dev(x), return_stats=True, seed=seed, **opts)
        assert np.array_equal(ids.numpy(), oids)
        _check(st, ost)
        for _ in range(2):   # the captured-graph path
            assert np.array_equal(sky.skyline(_dev(x), seed=seed, **opts).numpy(), oids)


def test_seed_changes_random_choices_not_the_skyline(sky, orc):
    x = datagen.anticorrelated(30_000, 5, 44)
    want = orc.sky_sfs(x)
    sizes = set()
    for seed in range(4):
        ids, st = sky.skyline(_dev(x), return_stats=True, seed=seed, partitioning="random", p=8, reps="random",
                              n_reps=32)
        assert np.array_equal(ids.numpy(), want)
        sizes.add(tuple(st["local_sizes"]))
    assert len(sizes) > 1


def test_sorted_part_full_size(sky, orc):
    """1M x 6 anticorrelated, Sliced p = 16, Sorted representatives taken per partition
    (4 per slice): ids, picks and every count equal the oracle's."""
    x = datagen.workload("sliced_ant_1m_d6")
    opts = dict(partitioning="sliced", p=16, reps="sorted_part", n_reps=64)
    oids, ost = orc.pipeline(x, threads=16, **opts)
    ids, st = sky.skyline(_dev(x), return_stats=True, **opts)
    assert np.array_equal(ids.numpy(), oids)
    _check(st, ost)
    assert np.array_equal(sky.skyline(_dev(x), **opts).numpy(), oids)


def test_sorted_part_limit(sky):
    x = _dev(datagen.anticorrelated(1000, 3, 46))
    with pytest.raises(sky.SkylineError) as e:   # 300 slices of one representative each
        sky.skyline(x, partitioning="sliced", p=300, reps="sorted_part", n_reps=64)
    assert e.value.code == -1


def test_region_needs_unit_range(sky):
    x = _dev(datagen.anticorrelated(1000, 3, 45) * 3.0)
    with pytest.raises(sky.SkylineError) as e:
        sky.skyline(x, partitioning="sliced", p=4, reps="region", n_reps=8)
    assert e.value.code == -3


def test_region_full_size(sky, orc):
    """1M x 6 anticorrelated, Sliced p = 16 with 64 Region representatives: exact."""
    x = datagen.workload("sliced_ant_1m_d6")
    opts = dict(partitioning="sliced", p=16, reps="region", n_reps=64)
    oids, ost = orc.pipeline(x, threads=16, **opts)
    ids, st = sky.skyline(_dev(x), return_stats=True, **opts)
    assert np.array_equal(ids.numpy(), oids)
    _check(st, ost)
