"""GPU parity of the batched skyline (many instances in one launch sequence).

Every instance's ids are compared bit-exactly with the oracle's skyline of that
instance alone: instances of mixed sizes (including 0, 1 and 2 points), mixed
dimensions (so several record widths), uniform, correlated, anticorrelated and
tie-heavy data, and every supported option set. The expected values come from
``oracle`` only.
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


def _instances():
    xs = datagen.batch_instances(n_inst=28, seed=11, n_lo=200, n_hi=6000)
    xs += [datagen.discrete(3000, 4, 5, 3), datagen.discrete(1500, 6, 6, 4),   # ties across slice boundaries
           datagen.uniform(0, 5, 1), datagen.uniform(1, 3, 2), datagen.uniform(2, 7, 3),
           datagen.anticorrelated(65, 2, 4), datagen.anticorrelated(2000, 1, 5),
           datagen.anticorrelated(3000, 11, 6)]
    return xs


@pytest.mark.parametrize("opts", [dict(), dict(p=7, n_reps=5), dict(p=1, reps="none"),
                                  dict(p=16, presort="sum"), dict(partitioning="none")])
def test_batch_matches_oracle(sky, orc, opts):
    xs = _instances()
    packed, ns, ds = sky.pack_instances([torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in xs])
    out, st = sky.skyline_batch(packed, ns, ds, return_stats=True, **opts)
    assert len(out) == len(xs)
    total = 0
    for x, ids in zip(xs, out):
        want = orc.sky_sfs(x) if x.shape[1] else np.zeros(0, np.int64)
        assert np.array_equal(ids.numpy(), want)
        total += len(want)
    assert st["size_sky"] == total and st["n_total"] == sum(ns)
    assert st["n_groups"] == len({(d + 2 + 3) // 4 for d, n in zip(ds, ns) if n})


def test_batch_errors(sky):
    x = torch.from_numpy(datagen.uniform(100, 3, 1)).cuda()
    packed, ns, ds = sky.pack_instances([x])
    for bad in (dict(partitioning="grid", p=8), dict(reps="learned"), dict(presort="learned")):
        with pytest.raises((sky.SkylineError, KeyError, ValueError)):
            sky.skyline_batch(packed, ns, ds, **bad)


def test_batch_full_size_sampled(sky, orc):
    """512 instances, sizes log-uniform in [1k, 200k], d uniform in {3..8}, uniform /
    correlated / anticorrelated at random (about 19M points): every instance's ids
    are ascending and inside the instance; instances that the oracle finishes quickly
    are compared exactly, the others by sampled skyline properties."""
    xs = datagen.batch_instances()
    packed, ns, ds = sky.pack_instances([torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in xs])
    out = sky.skyline_batch(packed, ns, ds)
    rng = np.random.default_rng(13)
    exact = [i for i in rng.permutation(len(xs)) if xs[i].shape[1] <= 20_000][:12]
    for i in exact:
        assert np.array_equal(out[i].numpy(), orc.sky_sfs(xs[i])), i
    for i in rng.choice(len(xs), 24, replace=False):
        x, ids = xs[i], out[i].numpy()
        assert len(ids) > 0 and np.all(np.diff(ids) > 0) and ids[-1] < x.shape[1]
        sk = x[:, ids]
        for t in rng.choice(ids, min(4, len(ids)), replace=False):
            p_ = x[:, t:t + 1]
            assert not ((x <= p_).all(0) & (x < p_).any(0)).any(), (i, t)
        rest = np.setdiff1d(rng.choice(x.shape[1], 64, replace=False), ids)[:8]
        for t in rest:
            p_ = x[:, t:t + 1]
            assert ((sk <= p_).all(0) & (sk < p_).any(0)).any(), (i, t)


def test_batch_first_call_on_fresh_context(sky, orc):
    """A batch as the very first call of a new context, after other contexts freed their
    workspace: every piece of device state the batch reads must be set by the batch itself
    (its radix sorts' scan ticket once was not)."""
    xs = [datagen.anticorrelated(n, d, 40 + i) for i, (n, d) in enumerate([(3000, 4), (800, 6), (2500, 7)])]
    for _ in range(2):
        c = sky.Context(0)
        try:
            x = torch.from_numpy(datagen.uniform(50_000, 6, 2)).cuda()
            sky.skyline(x, ctx=c)   # fills and frees a workspace
        finally:
            c.close()
    c = sky.Context(0)
    try:
        packed, ns, ds = sky.pack_instances([torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in xs])
        out = sky.skyline_batch(packed, ns, ds, p=5, ctx=c)
        for x, ids in zip(xs, out):
            assert np.array_equal(ids.numpy(), orc.sky_sfs(x))
    finally:
        c.close()


def test_batch_into_caller_buffer(sky, orc):
    xs = [datagen.correlated(1200, 3, 7), datagen.anticorrelated(900, 5, 8), datagen.uniform(0, 4, 1)]
    packed, ns, ds = sky.pack_instances([torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in xs])
    buf = torch.full((sum(ns) + 5,), -7, dtype=torch.int64)
    for _ in range(2):   # reused buffer
        out = sky.skyline_batch(packed, ns, ds, p=3, out=buf)
        for x, ids in zip(xs, out):
            want = orc.sky_sfs(x) if x.shape[1] else np.zeros(0, np.int64)
            assert np.array_equal(ids.numpy(), want)
            assert ids.numel() == 0 or ids.data_ptr() >= buf.data_ptr()
    with pytest.raises(ValueError):
        sky.skyline_batch(packed, ns, ds, out=torch.empty(3, dtype=torch.int64))
