"""GPU checks of the captured-graph path of sky_skyline.

A call without stats, phase times, work counts or a learned model replays a HIP
graph of its launch sequence. Every replay must equal the oracle's skyline: the
graph is replayed several times with other (eager) work and synchronisations in
between, on new data behind the same pointer, after the workspace grew (which
drops the graphs), with pinned and pageable output buffers, and on inputs whose
Sliced tie check fires (the graph assumes no tie, so the call reruns eagerly).
Expected values come from ``oracle`` only.
"""
import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sky():
    import paper_2411_14968_amd as m
    assert torch.cuda.is_available()
    return m


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


OPTS = [dict(partitioning="sliced", p=16),
        dict(partitioning="sliced", p=100, n_reps=16),                # rank-sort slices
        dict(partitioning="sliced", p=16, merge="global", presort="sum"),
        dict(partitioning="grid", p=16, m_per_dim=[2, 2, 2, 2], reps="none", grid_filter=True),
        dict(partitioning="angular", p=8, m_per_dim=[2, 2, 2]),
        dict(partitioning="none", reps="sorted", n_reps=8)]


@pytest.mark.parametrize("opts", OPTS)
def test_replays_match_oracle(sky, orc, opts):
    ctx = sky.Context(0)
    try:
        x = datagen.anticorrelated(40_000, 4, 5)
        other = datagen.correlated(7_000, 3, 6)
        want, want_o = orc.sky_sfs(x), orc.sky_sfs(other)
        xd, od = _dev(x), _dev(other)
        assert np.array_equal(sky.skyline(xd, ctx=ctx, graph=False, **opts).numpy(), want)
        for rep in range(4):
            ids = sky.skyline(xd, ctx=ctx, **opts)          # captured on the first pass, replayed after
            assert np.array_equal(ids.numpy(), want), rep
            # eager work of the program itself between the replays
            assert np.array_equal(sky.skyline(od, ctx=ctx, graph=False, p=4).numpy(), want_o)
            torch.cuda.synchronize()
            y = (xd * 2.0).sum()
            assert torch.isfinite(y)
    finally:
        ctx.close()


def test_new_data_same_pointer_and_growth(sky, orc):
    ctx = sky.Context(0)
    try:
        xs = [datagen.anticorrelated(30_000, 6, s) for s in (7, 8, 9)]
        buf = _dev(xs[0])
        for x in xs:   # same device pointer, new contents: the replay reads them
            buf.copy_(torch.from_numpy(x))
            assert np.array_equal(sky.skyline(buf, ctx=ctx).numpy(), orc.sky_sfs(x))
        big = datagen.anticorrelated(120_000, 6, 10)   # grows the workspace: graphs are dropped
        assert np.array_equal(sky.skyline(_dev(big), ctx=ctx).numpy(), orc.sky_sfs(big))
        buf.copy_(torch.from_numpy(xs[1]))
        for _ in range(2):
            assert np.array_equal(sky.skyline(buf, ctx=ctx).numpy(), orc.sky_sfs(xs[1]))
    finally:
        ctx.close()


def test_pinned_and_pageable_outputs(sky, orc):
    ctx = sky.Context(0)
    try:
        x = datagen.anticorrelated(25_000, 5, 11)
        want = orc.sky_sfs(x)
        xd = _dev(x)
        for out in (torch.empty(x.shape[1], dtype=torch.int64).pin_memory(),
                    torch.empty(x.shape[1], dtype=torch.int64)):
            for _ in range(3):
                out.fill_(-1)
                ids = sky.skyline(xd, ctx=ctx, out=out)
                assert np.array_equal(ids.numpy(), want)
    finally:
        ctx.close()


def test_tie_check_reruns_without_graph(sky, orc):
    """Few distinct values: equal x_s straddle slice boundaries, the graph's assumption
    fails and the call reruns eagerly (lexicographic slices)."""
    ctx = sky.Context(0)
    try:
        x = datagen.discrete(20_000, 4, 3, 3)
        opts = dict(partitioning="sliced", p=16, slice_dim=0, n_reps=16)
        oids, _ = orc.pipeline(x, threads=4, **opts)
        xd = _dev(x)
        for _ in range(3):
            assert np.array_equal(sky.skyline(xd, ctx=ctx, **opts).numpy(), oids)
    finally:
        ctx.close()


def test_learned_calls_replay_with_current_model(sky, orc):
    """Learned representatives and presort through the captured graph: the model is part of
    the key, its weights are read at each replay (training in between is seen), and a new
    model at possibly the same address gets a graph of its own."""
    ctx = sky.Context(0)
    try:
        d = 5
        x = datagen.anticorrelated(30_000, d, 12)
        want = orc.sky_sfs(x)
        xd = _dev(x)
        for round_ in range(2):
            m = sky.Scorer(d, seed=round_ + 3, ctx=ctx)
            for presort in ("zorder", "learned"):
                for _ in range(3):
                    ids = sky.skyline(xd, ctx=ctx, reps="learned", presort=presort, model=m, p=8)
                    assert np.array_equal(ids.numpy(), want), (round_, presort)
            # train a little: the replay reads the new weights
            y = torch.rand(x.shape[1], device="cuda")
            m.train(xd, y, epochs=1, batch=4096)
            for _ in range(2):
                assert np.array_equal(sky.skyline(xd, ctx=ctx, reps="learned", model=m, p=8).numpy(), want)
            del m
    finally:
        ctx.close()
