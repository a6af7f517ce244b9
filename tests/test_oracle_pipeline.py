"""Pins for the oracle's partitioning, filtering and Algorithm 2 pipeline.

* Grid cells (Section 3.2) on hand-computed points; Grid Filtering against the
  discard rate the paper prints for uniform data (Section 5.1) and its closed
  form (1 - 1/m)^d; soundness of every discarded point by brute force.
* Angular cells (Eq. (1)) against the angle formula evaluated with libm atan2,
  away from slice boundaries.
* Sliced sizes (Section 3.4) against the closed form ceil((j+1)N/p) - ceil(jN/p)
  and the order against numpy's lexsort.
* Sorted representatives against numpy's stable sort of float32 sums.
* Propositions 1 and 2 and representative soundness: every option combination
  returns the brute-force skyline; intermediate counts are recounted by brute force.
"""
import numpy as np
import pytest

import datagen


def test_grid_cells_hand_computed(orc):
    # dimension 0 is the least significant digit; x = 1.0 is clamped to m - 1
    x = np.array([[0.75, 0.25, 1.0, 0.0, 0.5], [0.25, 0.75, 1.0, 0.0, 0.49999997]], np.float32)
    assert orc.grid_cells(x, 2).tolist() == [1, 2, 3, 0, 1]
    assert orc.grid_cells(x, [4, 3]).tolist() == [3 + 4 * 0, 1 + 4 * 2, 3 + 4 * 2, 0, 2 + 4 * 1]
    with pytest.raises(ValueError):
        orc.grid_cells(np.array([[1.5], [0.2]], np.float32), 2)


def test_grid_filter_paper_rate_uniform(orc):
    """Section 5.1 reports 58% of uniform d=4 tuples discarded by Grid Filtering; the
    closed form (1 - 1/m)^4 gives 58.6% at m = 8 once the corner cell is occupied."""
    x = datagen.uniform(200_000, 4, 11)
    pr = orc.grid_filter(x, 8)
    assert abs(pr.mean() - (7 / 8) ** 4) < 0.005
    assert abs(pr.mean() - 0.58) < 0.01


def test_grid_filter_m2_exact_set(orc):
    """With m = 2 and cell 0 occupied the discarded points are exactly those with
    every coordinate >= 0.5."""
    x = datagen.uniform(10_000, 4, 1)
    pr = orc.grid_filter(x, 2)
    assert np.array_equal(pr, (x >= 0.5).all(axis=0))


@pytest.mark.parametrize("seed", range(4))
def test_grid_filter_sound(orc, seed):
    x = datagen.discrete(800, 3, seed, 9)
    pr = orc.grid_filter(x, [3, 4, 2])
    sky = set(orc.sky_brute(x).tolist())
    assert not any(i in sky for i in np.flatnonzero(pr))


def test_angular_matches_atan(orc):
    rng = np.random.default_rng(3)
    for d, m in ((2, [5]), (3, [4, 3]), (4, [2, 3, 2]), (8, [2] * 6 + [1])):
        x = rng.random((d, 5000)).astype(np.float32)
        got = orc.angular_cells(x, m)
        xd = x.astype(np.float64)
        want = np.zeros(x.shape[1], np.int64)
        near = np.zeros(x.shape[1], bool)
        mult = 1
        for i in range(d - 1):
            rest = np.sqrt((xd[i + 1:] ** 2).sum(0))
            phi = np.arctan2(rest, xd[i])
            v = 2 * phi * m[i] / np.pi
            digit = np.minimum(np.floor(v), m[i] - 1).astype(np.int64)
            near |= np.abs(v - np.round(v)) < 1e-9
            want += digit * mult
            mult *= m[i]
        assert np.array_equal(got[~near], want[~near])
        assert (~near).mean() > 0.99


def test_angular_axes(orc):
    # x_1 = 0 gives phi_1 = pi/2, clamped to the last slice; a point on the first
    # axis gives phi = 0; the origin (0/0) falls into the last slice.
    x = np.array([[0.0, 0.7, 0.0], [0.5, 0.0, 0.0]], np.float32)
    assert orc.angular_cells(x, [4]).tolist() == [3, 0, 3]


@pytest.mark.parametrize("n,p", [(10_000, 16), (1001, 7), (5, 16), (64, 64), (100, 1)])
def test_sliced_sizes_closed_form(orc, n, p):
    x = datagen.uniform(n, 3, n + p)
    c = orc.sliced_cells(x, p, 1)
    sizes = np.bincount(c, minlength=p)
    j = np.arange(p)
    # rank r goes to floor(r p / N), so slice j holds ranks in [jN/p, (j+1)N/p)
    ceil = lambda a: -(-a // p)
    assert np.array_equal(sizes, ceil((j + 1) * n) - ceil(j * n))


def test_sliced_order_lexicographic(orc):
    """Ties on the slicing dimension are broken by the other coordinates, then by id."""
    x = datagen.discrete(3000, 4, 8, 3)
    s = 2
    c = orc.sliced_cells(x, 10, s)
    keys = [np.arange(x.shape[1])] + [x[k] for k in reversed(range(4)) if k != s] + [x[s]]
    order = np.lexsort(tuple(keys))
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    assert np.array_equal(c, rank * 10 // x.shape[1])


def test_sorted_reps(orc):
    x = datagen.discrete(5000, 5, 4, 50)
    sc = orc.sum_scores(x)
    acc = x[0].copy()
    for k in range(1, 5):
        acc = (acc + x[k]).astype(np.float32)
    assert np.array_equal(sc, acc)
    ids = orc.select_reps(sc, 64)
    assert np.array_equal(ids, np.argsort(sc, kind="stable")[:64])
    keep = orc.rep_selfilter(x, ids)
    sky_of_reps = orc.sky_brute(x[:, ids])
    assert np.array_equal(np.flatnonzero(keep), sky_of_reps)


def _combos():
    out = []
    for part, p, m in (("none", 1, None), ("grid", 8, [2, 2, 2]), ("grid", 12, [3, 2, 2]),
                       ("angular", 6, [3, 2]), ("angular", 1, [1, 1]), ("sliced", 1, None),
                       ("sliced", 3, None), ("sliced", 16, None), ("sliced", 64, None)):
        for reps in ("none", "sorted", "scores"):
            for merge in ("noseq", "global"):
                for gf in (False, True):
                    out.append(pytest.param(part, p, m, reps, merge, gf,
                                            id=f"{part}{p}-{reps}-{merge}-gf{int(gf)}"))
    return out


@pytest.mark.parametrize("part,p,m,reps,merge,gf", _combos())
def test_pipeline_equals_definition(orc, part, p, m, reps, merge, gf):
    """Propositions 1 and 2 and representative soundness: every option set gives Sky(r)."""
    for x in (datagen.discrete(700, 3, 21, 5), datagen.anticorrelated(700, 3, 22)):
        want = orc.sky_brute(x)
        scores = np.random.default_rng(1).random(x.shape[1]).astype(np.float32)
        ids, st = orc.pipeline(x, partitioning=part, p=p, m_per_dim=m, reps=reps, n_reps=16,
                               scores=scores, grid_filter=gf, grid_filter_m=3, merge=merge,
                               threads=2)
        assert np.array_equal(ids, want)
        assert st["size_sky"] == want.size


def test_pipeline_statistics_recount(orc):
    x = datagen.anticorrelated(3000, 4, 5)
    ids, st = orc.pipeline(x, partitioning="sliced", p=8, reps="sorted", n_reps=32)
    n = x.shape[1]
    sc = orc.sum_scores(x)
    reps = np.argsort(sc, kind="stable")[:32]
    assert np.array_equal(st["rep_ids"], reps)
    kept = reps[orc.rep_selfilter(x, reps)]
    assert st["n_reps_kept"] == kept.size
    # survivors: not dominated by any kept representative (vectorised recount)
    T = x[:, kept][:, :, None]
    S = x[:, None, :]
    dom = (((T <= S).all(0)) & ((T < S).any(0))).any(0)
    alive = ~dom
    assert st["n_after_reps"] == alive.sum()
    part = orc.sliced_cells(x, 8, 0)
    assert np.array_equal(st["part_sizes"], np.bincount(part, minlength=8))
    assert np.array_equal(st["part_kept"], np.bincount(part[alive], minlength=8))
    for j in range(8):
        mem = np.flatnonzero(alive & (part == j))
        assert st["local_sizes"][j] == orc.sky_brute(x[:, mem]).size
    assert st["size_u"] == st["local_sizes"].sum()
    assert np.array_equal(ids, orc.sky_brute(x))


def test_pipeline_threads_and_ties(orc):
    x = datagen.mixture_quantized(20_000, 5, 3)
    a, sa = orc.pipeline(x, partitioning="angular", p=16, m_per_dim=[2, 2, 2, 2], grid_filter=True,
                         grid_filter_m=4, reps="sorted", threads=1)
    b, sb = orc.pipeline(x, partitioning="angular", p=16, m_per_dim=[2, 2, 2, 2], grid_filter=True,
                         grid_filter_m=4, reps="sorted", threads=4, merge="global")
    assert np.array_equal(a, b)
    assert np.array_equal(a, orc.sky_sfs(x))
    assert sa["local_sizes"].tolist() == sb["local_sizes"].tolist()


def test_pipeline_rejects(orc):
    x = datagen.uniform(50, 3, 1)
    with pytest.raises(ValueError):
        orc.pipeline(x, partitioning="grid", p=9, m_per_dim=[2, 2, 2])      # p != prod m
    with pytest.raises(ValueError):
        orc.pipeline(x * 2, partitioning="grid", p=8, m_per_dim=[2, 2, 2])  # outside [0,1]
