"""GPU checks of the dominance kernels' work splits and the autotuner.

Every split must leave the result unchanged: the skyline is compared bit-exactly
with the oracle's under the extreme values of each field (points per lane 1, 2
and 4 for every record width, so live points packed into 1 to 4 rows, segments of 256 and 8192 records, 1 and 8 workgroups per
compute unit), for the local kernel, the NoSeq merge and the final round. The
tuning table's set / get / save / load round trip and its error cases, and the
autotuner's contract (valid splits, never slower than where it started, the
result unchanged) are checked as well. Expected values come from ``oracle`` only.
"""
import os

import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu

SPLITS = [
    dict(local_ppl=1, local_seg=256, merge_ppl=1, merge_seg=256, wg_per_cu=1),
    dict(local_ppl=2, local_seg=8192, merge_ppl=2, merge_seg=8192, wg_per_cu=8),
    dict(local_ppl=1, local_seg=4096, merge_ppl=2, merge_seg=256, wg_per_cu=4),
    dict(local_ppl=2, local_seg=256, merge_ppl=1, merge_seg=2048, wg_per_cu=2),
    dict(local_ppl=4, local_seg=1024, merge_ppl=4, merge_seg=512, wg_per_cu=4),
    dict(local_ppl=4, local_seg=256, merge_ppl=4, merge_seg=8192, wg_per_cu=8),
]


@pytest.fixture(scope="module")
def sky():
    import paper_2411_14968_amd as m
    assert torch.cuda.is_available()
    return m


@pytest.fixture()
def ctx(sky):
    c = sky.Context(0)
    yield c
    c.close()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("case", [
    ("anti", 6, dict(p=16)),
    ("anti", 6, dict(p=16, merge="global")),
    ("anti", 10, dict(p=8)),                     # record width 12
    ("anti", 16, dict(p=4, reps="none")),         # record width 20
    ("tie", 4, dict(p=7, presort="sum")),
    ("anti", 3, dict(partitioning="angular", p=4, m_per_dim=[2, 2])),
    ("anti", 4, dict(partitioning="grid", p=16, m_per_dim=[2] * 4, reps="none")),
])
def test_every_split_matches_oracle(sky, orc, ctx, case):
    kind, d, opts = case
    n = 20_000 if d <= 6 else 5_000
    x = datagen.anticorrelated(n, d, 100 + d) if kind == "anti" else datagen.discrete(n, d, 6, 5)
    want = orc.sky_sfs(x)
    xd = _dev(x)
    for split in SPLITS:
        sky.tune_set(d, n, split, ctx=ctx)
        assert sky.tune_get(d, n, ctx=ctx) == (split, True)
        ids = sky.skyline(xd, ctx=ctx, **opts)
        assert np.array_equal(ids.numpy(), want), split


def test_batch_split_matches_oracle(sky, orc, ctx):
    xs = datagen.batch_instances(n_inst=24, seed=5, n_lo=300, n_hi=5000)
    packed, ns, ds = sky.pack_instances([_dev(x) for x in xs])
    groups = {}
    for n, d in zip(ns, ds):
        dp = (d + 2 + 3) // 4 * 4
        groups.setdefault(dp, [0, d])[0] += n
    for split in SPLITS[:2]:
        for dp, (nt, d) in groups.items():
            sky.tune_set(d, nt, split, ctx=ctx)
        out = sky.skyline_batch(packed, ns, ds, p=5, ctx=ctx)
        for x, ids in zip(xs, out):
            assert np.array_equal(ids.numpy(), orc.sky_sfs(x))


def test_table_roundtrip_and_errors(sky, ctx, tmp_path):
    base = sky.tune_default(6)
    assert sky.tune_get(6, 5000, ctx=ctx) == (base, False)
    sky.tune_set(6, 5000, SPLITS[0], ctx=ctx)
    # one entry per (record width, floor(log2 n)): d = 5 shares width 8, 4096 <= n < 8192 shares the bucket
    assert sky.tune_get(5, 4096, ctx=ctx) == (SPLITS[0], True)
    assert sky.tune_get(6, 8192, ctx=ctx) == (base, False)
    sky.tune_set(12, 1 << 20, SPLITS[2], ctx=ctx)
    path = str(tmp_path / "tune.txt")
    sky.tune_save(path, ctx=ctx)
    lines = open(path).read().split("\n")
    assert lines[0].startswith("skyline-tune 1 gfx")
    assert sorted(lines[1:-1]) == ["16 20 1 4096 2 256 4", "8 12 1 256 1 256 1"]
    sky.tune_clear(ctx=ctx)
    assert sky.tune_get(6, 5000, ctx=ctx)[1] is False
    sky.tune_load(path, ctx=ctx)
    assert sky.tune_get(6, 5000, ctx=ctx) == (SPLITS[0], True)
    assert sky.tune_get(12, (1 << 20) + 5, ctx=ctx) == (SPLITS[2], True)
    # a table from another device, a malformed entry and a missing file leave the table unchanged
    magic, ver, arch, ncu = lines[0].split()
    other = str(tmp_path / "other.txt")
    with open(other, "w") as f:
        f.write("\n".join([f"{magic} {ver} gfx000 {ncu}"] + lines[1:]))
    fewer = str(tmp_path / "fewer.txt")
    with open(fewer, "w") as f:
        f.write("\n".join([f"{magic} {ver} {arch} {int(ncu) // 2}"] + lines[1:]))
    bad = str(tmp_path / "bad.txt")
    with open(bad, "w") as f:
        f.write(lines[0] + "\n8 3 3 1024 2 1024 8\n")
    trunc = str(tmp_path / "trunc.txt")
    with open(trunc, "w") as f:
        f.write(lines[0] + "\n8 3 1 1024\n")
    for p, code in ((other, -1), (fewer, -1), (bad, -1), (trunc, -1), (str(tmp_path / "none.txt"), -8)):
        with pytest.raises(sky.SkylineError) as e:
            sky.tune_load(p, ctx=ctx)
        assert e.value.code == code
    assert sky.tune_get(6, 5000, ctx=ctx) == (SPLITS[0], True)
    for badsplit in (dict(SPLITS[0], local_ppl=3), dict(SPLITS[0], local_seg=1000),
                     dict(SPLITS[0], merge_seg=128), dict(SPLITS[0], wg_per_cu=9)):
        with pytest.raises(sky.SkylineError):
            sky.tune_set(6, 5000, badsplit, ctx=ctx)


def test_autotune_contract(sky, orc, ctx):
    x = datagen.anticorrelated(60_000, 6, 21)
    want = orc.sky_sfs(x)
    xd = _dev(x)
    r = sky.autotune(xd, trials=3, ctx=ctx, p=16)
    assert r["best_ms"] > 0 and r["best_ms"] <= r["base_ms"]
    assert sky.tune_get(6, 60_000, ctx=ctx) == (r["params"], True)
    assert np.array_equal(sky.skyline(xd, ctx=ctx, p=16).numpy(), want)


def test_autotune_batch_contract(sky, orc, ctx):
    xs = datagen.batch_instances(n_inst=16, seed=9, n_lo=500, n_hi=4000)
    packed, ns, ds = sky.pack_instances([_dev(x) for x in xs])
    r = sky.autotune_batch(packed, ns, ds, trials=2, ctx=ctx, p=4)
    assert r["best_ms"] <= r["base_ms"]
    out = sky.skyline_batch(packed, ns, ds, p=4, ctx=ctx)
    for x, ids in zip(xs, out):
        assert np.array_equal(ids.numpy(), orc.sky_sfs(x))
