"""GPU parity of the skyline path against the CPU oracle.

Bit-exact comparison of index sets (dominance is a pure comparison, so no
tolerance applies) and of every count of Algorithm 2 (Grid Filtering,
representatives, partition sizes, local skyline sizes, |u|), over the
workloads' shapes, ragged sizes around the chunk size, ties and duplicates,
and every option combination. The expected values come from ``oracle`` only.
"""
import os

import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def sky():
    import paper_2411_14968_amd as m
    assert torch.cuda.is_available()
    return m


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _gpu(sky, x, **kw):
    ids, st = sky.skyline(_dev(x), return_stats=True, **kw)
    return ids.numpy(), st


def _check_stats(st, ost, np_):
    assert st["n_after_grid"] == ost["n_after_grid"]
    assert st["n_after_reps"] == ost["n_after_reps"]
    assert st["size_u"] == ost["size_u"]
    assert st["size_sky"] == ost["size_sky"]
    assert st["part_sizes"] == ost["part_sizes"].tolist()
    assert st["part_kept"] == ost["part_kept"].tolist()
    assert st["local_sizes"] == ost["local_sizes"].tolist()
    if "rep_ids" in ost:
        assert st["rep_ids"] == ost["rep_ids"].tolist()
        assert st["rep_keep"] == ost["rep_keep"].tolist()
        assert st["n_reps_kept"] == ost["n_reps_kept"]


def test_grid_uniform_10k_d4(sky, orc):
    """10,000 uniform points, d = 4, Grid with m = 2 (p = 16), with and without Grid Filtering."""
    x = datagen.workload("grid_uniform_10k_d4")
    want = orc.sky_brute(x)
    for gf in (False, True):
        opts = dict(partitioning="grid", p=16, m_per_dim=[2] * 4, reps="none", grid_filter=gf, merge="noseq")
        ids, st = _gpu(sky, x, **opts)
        assert np.array_equal(ids, want)
        oids, ost = orc.pipeline(x, threads=THREADS, **opts)
        assert np.array_equal(oids, want)
        _check_stats(st, ost, 16)
        if gf:   # m = 2, cell 0 occupied: exactly the points with every coordinate >= 0.5 go
            assert st["n_after_grid"] == 10_000 - int((x >= 0.5).all(axis=0).sum())


@pytest.mark.parametrize("n", [20_000, 1_000_000])
def test_sliced_anticorrelated_d6(sky, orc, n):
    """Anticorrelated d = 6, Sliced p = 16 on dimension 0, 64 Sorted representatives, NoSeq."""
    x = datagen.workload("sliced_ant_1m_d6", n=n)
    opts = dict(partitioning="sliced", p=16, reps="sorted", n_reps=64, merge="noseq")
    ids, st = _gpu(sky, x, **opts)
    oids, ost = orc.pipeline(x, threads=THREADS, **opts)
    assert np.array_equal(ids, oids)
    _check_stats(st, ost, 16)
    if n <= 20_000:
        assert np.array_equal(ids, orc.sky_brute(x))


def _opt_sets(d):
    out = [dict(partitioning="none", reps="none"),
           dict(partitioning="none", reps="sorted", n_reps=16),
           dict(partitioning="sliced", p=1, reps="none"),
           dict(partitioning="sliced", p=7, reps="sorted", n_reps=5, merge="noseq", presort="sum"),
           dict(partitioning="sliced", p=16, reps="sorted", n_reps=64, merge="global"),
           dict(partitioning="sliced", p=3, reps="none", grid_filter=True, grid_filter_m=3),
           dict(partitioning="grid", p=2 ** d, m_per_dim=[2] * d, reps="none", grid_filter=True),
           dict(partitioning="grid", p=3 ** min(d, 2), m_per_dim=[3] * min(d, 2) + [1] * (d - min(d, 2)),
                reps="sorted", n_reps=8, merge="global", presort="sum")]
    if d >= 2:
        out += [dict(partitioning="angular", p=2 ** (d - 1), m_per_dim=[2] * (d - 1), reps="sorted", n_reps=32),
                dict(partitioning="angular", p=3, m_per_dim=[3] + [1] * (d - 2), reps="none", merge="global",
                     grid_filter=True, grid_filter_m=2)]
    return out


@pytest.mark.parametrize("d", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("n", [0, 1, 2, 65, 1023, 1024, 1025, 3000])
def test_option_sweep(sky, orc, d, n):
    """Every option set gives the skyline (Propositions 1 and 2) with oracle-equal counts,
    on ragged sizes around the chunk size and with heavy ties."""
    for levels in (0, 4):
        x = datagen.discrete(n, d, 7 * n + d, levels) if levels else datagen.anticorrelated(n, d, n + d) \
            if d > 1 else datagen.uniform(n, d, n)
        want = orc.sky_brute(x)
        for opts in _opt_sets(d):
            if opts["partitioning"] == "grid" and 2 ** d > 65536:
                continue
            ids, st = _gpu(sky, x, **opts)
            assert np.array_equal(ids, want), opts
            if n:
                oids, ost = orc.pipeline(x, threads=1, **opts)
                _check_stats(st, ost, opts.get("p", 1))


@pytest.mark.parametrize("d", [11, 16])
def test_high_dimensions(sky, orc, d):
    x = datagen.anticorrelated(4000, d, d)
    want = orc.sky_sfs(x)
    for opts in (dict(partitioning="sliced", p=8, reps="sorted", n_reps=64),
                 dict(partitioning="none", reps="none"),
                 dict(partitioning="angular", p=2, m_per_dim=[2] + [1] * (d - 2), reps="sorted", merge="global")):
        ids, _ = _gpu(sky, x, **opts)
        assert np.array_equal(ids, want)


def test_special_cases(sky, orc):
    # all-equal: every id
    x = np.full((4, 3000), 0.25, np.float32)
    assert np.array_equal(sky.skyline(_dev(x)).numpy(), np.arange(3000))
    # chain with two copies of the minimum
    v = (np.arange(5000) / 5000 * 0.8 + 0.1).astype(np.float32)
    v[17] = v[4000] = 0.0
    x = np.tile(v, (3, 1))
    for opts in (dict(), dict(partitioning="grid", p=8, m_per_dim=[2, 2, 2], reps="none"),
                 dict(partitioning="angular", p=4, m_per_dim=[2, 2])):
        assert sky.skyline(_dev(x), **opts).tolist() == [17, 4000]
    # antichain on x + y = 1
    t = np.linspace(0, 1, 4097, dtype=np.float32)
    x = np.stack([t, (1 - t).astype(np.float32)])
    assert np.array_equal(sky.skyline(_dev(x)).numpy(), orc.sky_2d(x))
    # d = 1
    x = datagen.discrete(5000, 1, 3, 20)
    assert np.array_equal(sky.skyline(_dev(x), reps="sorted").numpy(), np.flatnonzero(x[0] == x[0].min()))
    # duplicates share one fate; negative zero equals zero
    base = datagen.anticorrelated(3000, 5, 4)
    x = np.concatenate([base, base[:, :700]], axis=1)
    x[2, 5] = -0.0
    ids = sky.skyline(_dev(x), partitioning="sliced", p=16).numpy()
    assert np.array_equal(ids, orc.sky_brute(x))
    # negative and large finite values (no range requirement for Sliced / none)
    y = (datagen.anticorrelated(2000, 3, 5) - 0.5) * 1e30
    assert np.array_equal(sky.skyline(_dev(y)).numpy(), orc.sky_brute(y))
    # a range wider than the largest float (the Z-order scale degenerates to 0)
    y = ((datagen.anticorrelated(2000, 3, 6).astype(np.float64) - 0.5) * 6.6e38).astype(np.float32)
    with np.errstate(over="ignore"):   # the float32 range overflows on purpose
        assert np.isfinite(y).all() and y.max() - y.min() == np.inf
    assert np.array_equal(sky.skyline(_dev(y)).numpy(), orc.sky_brute(y))
    # one coordinate constant
    y = datagen.anticorrelated(3000, 4, 8)
    y[1] = 0.5
    assert np.array_equal(sky.skyline(_dev(y), p=8).numpy(), orc.sky_brute(y))


@pytest.mark.parametrize("presort", ["zorder", "sum", "zorder_sum"])
def test_presort_orders(sky, orc, presort):
    """The SFS presort order (Z-order or coordinate sum) changes the work, never the
    result: skyline and every count equal the oracle's, for NoSeq and the global merge."""
    x = datagen.workload("sliced_ant_1m_d6", n=200_000)
    for merge in ("noseq", "global"):
        opts = dict(partitioning="sliced", p=16, reps="sorted", n_reps=64, merge=merge)
        ids, st = _gpu(sky, x, presort=presort, **opts)
        oids, ost = orc.pipeline(x, threads=THREADS, **opts)
        assert np.array_equal(ids, oids)
        _check_stats(st, ost, 16)


@pytest.mark.parametrize("d", [7, 8, 12])
def test_wide_zorder_key(sky, orc, d):
    """From d = 7 the Z-order presort sorts a 64-bit key (partition bits, then 7 to 9 bits
    per coordinate): one partition, where the code fills the whole word, 120 Sliced
    partitions and 64 Angular ones, on continuous data and on data full of duplicates.
    Exact against the oracle with every count, and the same set under the sum orders."""
    for x in (datagen.anticorrelated(60_000, d, 70 + d), datagen.discrete(60_000, d, 80 + d, 5)):
        for opts in (dict(partitioning="none", reps="none"),
                     dict(partitioning="sliced", p=120, reps="sorted", n_reps=64, merge="noseq"),
                     dict(partitioning="angular", p=64, m_per_dim=[2] * 6 + [1] * (d - 7), reps="sorted",
                          n_reps=64, merge="global")):
            ids, st = _gpu(sky, x, presort="zorder", **opts)
            oids, ost = orc.pipeline(x, threads=THREADS, **opts)
            assert np.array_equal(ids, oids), opts
            _check_stats(st, ost, opts.get("p", 1))
            for presort in ("zorder_sum", "sum"):
                assert np.array_equal(_gpu(sky, x, presort=presort, **opts)[0], oids), (presort, opts)


@pytest.mark.parametrize("reps", ["sorted", "sorted_part"])
def test_sliced_ties_across_boundaries(sky, orc, reps):
    """Few distinct values on the slicing dimension: runs of equal x_s straddle slice
    boundaries, so the lexicographic tie-break decides the slices (also when the
    representatives are taken per partition, after the slices are final)."""
    x = datagen.discrete(20_000, 4, 3, 3)
    for s in (0, 2):
        opts = dict(partitioning="sliced", p=16, slice_dim=s, reps=reps, n_reps=16)
        ids, st = _gpu(sky, x, **opts)
        oids, ost = orc.pipeline(x, threads=THREADS, **opts)
        assert np.array_equal(ids, oids)
        _check_stats(st, ost, 16)


@pytest.mark.parametrize("reps", ["sorted", "none"])
@pytest.mark.parametrize("p", [2, 17, 63, 64, 65, 300])
def test_sliced_boundaries_selected_or_sorted(sky, orc, p, reps):
    """Up to 64 slices the slice boundaries come from a radix selection (the filter assigns
    the slices); more slices use the rank sort. Both must give the oracle's slices: inputs
    with clipped (tied) values that do not straddle a boundary, ties that do, fewer points
    than slices, and a single point. With representatives the selection's passes run inside
    their select launches; without, in launches of their own."""
    cases = [(datagen.anticorrelated(30_000, 5, 17), 0), (datagen.correlated(20_000, 4, 18), 3),
             (datagen.discrete(5_000, 3, 19, 4), 1), (datagen.uniform(p // 2 + 1, 4, 20), 0),
             (datagen.uniform(1, 3, 21), 2)]
    for x, sd in cases:
        opts = dict(partitioning="sliced", p=p, slice_dim=sd, reps=reps)
        if reps != "none":
            opts["n_reps"] = 16
        ids, st = _gpu(sky, x, **opts)
        oids, ost = orc.pipeline(x, threads=THREADS, **opts)
        assert np.array_equal(ids, oids), (x.shape, sd)
        _check_stats(st, ost, p)


def test_mixture_quantized_angular(sky, orc):
    """Clustered + anticorrelated, 1000 levels (exact duplicates), Angular p = 64 on d = 8
    with Grid Filtering m_g = 4, at 200k points."""
    x = datagen.workload("angular_mix_10m_d8", n=200_000)
    for merge in ("global", "noseq"):
        opts = dict(partitioning="angular", p=64, m_per_dim=[2, 2, 2, 2, 2, 2, 1], grid_filter=True,
                    grid_filter_m=4, reps="sorted", n_reps=64, merge=merge)
        ids, st = _gpu(sky, x, **opts)
        oids, ost = orc.pipeline(x, threads=THREADS, **opts)
        assert np.array_equal(ids, oids)
        _check_stats(st, ost, 64)


def test_deterministic(sky):
    x = _dev(datagen.workload("sliced_ant_1m_d6", n=200_000))
    ref, st0 = sky.skyline(x, return_stats=True)
    for _ in range(4):
        ids, st = sky.skyline(x, return_stats=True)
        assert torch.equal(ids, ref)
        st.pop("ms_total"), st0.pop("ms_total", None)
        assert st == st0


def test_work_counts(sky):
    """The instrumented call returns the same skyline and plausible work counts: whole
    query-group multiples, corner checks present, nothing for an empty input."""
    x = _dev(datagen.workload("sliced_ant_1m_d6", n=200_000))
    ref = sky.skyline(x)
    ids, st = sky.skyline(x, return_stats=True, count_work=True)
    assert torch.equal(ids, ref)
    w = st["work"]
    assert w["local_tests"] > 0 and w["merge_tests"] > 0
    assert w["local_corner_checks"] > 0 and w["merge_corner_checks"] > 0
    assert w["local_tests"] % 64 == 0 and w["merge_tests"] % 64 == 0
    assert 0 < w["local_alive_tests"] <= w["local_tests"] and 0 < w["merge_alive_tests"] <= w["merge_tests"]
    assert st["tests"] == w["local_alive_tests"] + w["merge_alive_tests"]
    _, st0 = sky.skyline(x, return_stats=True)
    assert all(v == 0 for v in st0["work"].values())


def test_errors(sky):
    x = datagen.uniform(1000, 3, 1)
    bad = x.copy()
    bad[1, 10] = np.nan
    with pytest.raises(sky.SkylineError) as e:
        sky.skyline(_dev(bad))
    assert e.value.code == -2
    bad[1, 10] = np.inf
    with pytest.raises(sky.SkylineError) as e:
        sky.skyline(_dev(bad), partitioning="none")
    assert e.value.code == -2
    with pytest.raises(sky.SkylineError) as e:
        sky.skyline(_dev(x * 2), partitioning="grid", p=8, m_per_dim=[2, 2, 2])
    assert e.value.code == -3
    with pytest.raises(sky.SkylineError) as e:
        sky.skyline(_dev(x), partitioning="grid", p=9)
    assert e.value.code == -1
    with pytest.raises(sky.SkylineError) as e:
        sky.skyline(_dev(x), reps="learned")
    assert e.value.code == -7
    # output capacity: the C-ABI returns SKY_ERR_CAPACITY and the size needed
    import ctypes as C
    t = np.linspace(0, 1, 100, dtype=np.float32)
    anti = _dev(np.stack([t, (1 - t).astype(np.float32)]))
    o = sky.make_opts()
    out = torch.empty(50, dtype=torch.int64)
    nout = C.c_int64(0)
    rc = sky.lib().sky_skyline(sky.context().h, C.c_void_p(anti.data_ptr()), 100, 2, C.byref(o),
                               C.c_void_p(out.data_ptr()), 50, C.byref(nout), None, None)
    assert rc == -4 and nout.value == 100
    with pytest.raises(ValueError):
        sky.skyline(anti, out=torch.empty(50, dtype=torch.int64))
    # the context stays usable after errors
    assert sky.skyline(_dev(x)).numel() > 0


@pytest.mark.parametrize("opts", [dict(partitioning="sliced", p=2400, reps="sorted", n_reps=64),
                                  dict(partitioning="sliced", p=600, reps="none", presort="sum"),
                                  dict(partitioning="angular", p=125, m_per_dim=[5, 5, 5], reps="sorted", n_reps=64),
                                  dict(partitioning="random", p=1200, reps="none", seed=3)])
def test_many_partitions_noseq(sky, orc, opts):
    """NoSeq with many small partitions, where the merge deals its work over one contiguous
    candidate range per query group (every earlier slice; every partition) instead of one
    item per candidate partition: the skyline and every count equal the oracle's."""
    x = datagen.anticorrelated(200_000, 4, 77)
    ids, st = _gpu(sky, x, merge="noseq", **opts)
    oids, ost = orc.pipeline(x, threads=THREADS, merge="noseq", **opts)
    assert np.array_equal(ids, oids)
    _check_stats(st, ost, opts["p"])
    assert np.array_equal(sky.skyline(_dev(x), merge="noseq", **opts).numpy(), oids)   # the captured graph


@pytest.mark.parametrize("name,opts", [
    ("HOU-shaped", dict(partitioning="grid", p=128, m_per_dim=[2] * 7, reps="none", merge="global")),
    ("HOU-shaped", dict(partitioning="sliced", p=16, reps="sorted", n_reps=64)),
    ("RES-shaped", dict(partitioning="angular", p=64, m_per_dim=[2] * 6, reps="sorted", n_reps=64)),
    ("RES-shaped", dict(partitioning="sliced", p=16, reps="sorted_part", n_reps=64))])
def test_tie_heavy_inputs(sky, orc, name, opts):
    """Inputs shaped like the paper's real datasets (readings on fixed steps, skewed
    spreads, zero-inflated attributes), 300k points: many points share a Z-order cell
    even under the 64-bit key of d = 7; also the narrow Z-order key, the key with the
    sum word and the sum order on a 6-dimensional projection. Exact against the
    oracle, with every count."""
    gen, _, d, seed = datagen.REAL_SHAPED[name]
    x = datagen.generate(gen, 300_000, d, seed)
    ids, st = _gpu(sky, x, **opts)
    oids, ost = orc.pipeline(x, threads=THREADS, **opts)
    assert np.array_equal(ids, oids)
    _check_stats(st, ost, opts["p"])
    x6 = np.ascontiguousarray(x[:6])
    o6 = dict(partitioning="sliced", p=16, reps="sorted", n_reps=64)
    want6, _ = orc.pipeline(x6, threads=THREADS, **o6)
    for presort in ("zorder", "zorder_sum", "sum"):
        assert np.array_equal(sky.skyline(_dev(x6), presort=presort, **o6).numpy(), want6), presort
