"""Pins for the oracle's representative rules, reverse counts, training targets and
work counters.

* Learned representatives: a hand-computed 2-D pool and mix (every coverage count
  worked out on paper), the duplicate rule of the pool, the reduction to Sorted
  representatives when the learned score is the sum itself, and the pipeline's
  skyline against brute force under the rule.
* Sorted representatives per partition (Section 4.1, the first tuples of each
  partition after sorting): a hand-computed case and numpy's stable sort per part.
* Reverse dominance counts: a hand case; over all points, "dominated by someone"
  is exactly "not in the skyline" (the brute-force definition); the totals of the
  forward and reverse counts over the same pairs agree.
* Training targets: y = 0 for a point that dominates nothing, y = -1 for one that
  dominates the whole sample, the residual sample recounted by brute force.
* Work counters: a 6-point input whose SFS comparisons and NoSeq merge comparisons
  are counted by hand (Algorithm 1; Proposition 2 with the key cutoff).
"""
import numpy as np
import pytest

import datagen


def _dominates(A, B):
    """[len(A), len(B)] bool: column a of A dominates column b of B (Def. 1)."""
    return (A[:, :, None] <= B[:, None, :]).all(0) & (A[:, :, None] < B[:, None, :]).any(0)


# ----------------------------------------------------------------- learned pool and mix
# Eight 2-D points (ids 0..7): A, B sit near the x-axis origin corner with the two
# smallest sums; C, D have the two smallest learned scores; E..H are the rest.
_PTS = np.array([
    [0.05, 0.06, 0.5, 0.3, 0.7, 0.8, 0.4, 0.9],     # x
    [0.5, 0.52, 0.1, 0.35, 0.6, 0.2, 0.9, 0.15],     # y
], np.float32)
A, B, Cc, D, E, F, G, H = range(8)
_LEARNED = np.array([0.3, 0.4, 0.1, 0.2, 0.9, 0.8, 0.7, 0.6])


def test_learned_pool_hand(orc):
    # sums: A .55, B .58, C .6, D .65, F 1.0, H 1.05, E 1.3, G 1.3
    pool = orc.learned_pool(orc.sum_scores(_PTS), _LEARNED, half=2)
    assert pool.tolist() == [A, B, Cc, D]
    # a learned candidate already among the sum candidates leaves its slot empty
    lsc = _LEARNED.copy()
    lsc[B] = 0.0
    assert orc.learned_pool(orc.sum_scores(_PTS), lsc, half=2).tolist() == [A, B, -1, Cc]
    # slots past n are empty in both halves (here every learned candidate is a sum one too)
    small = _PTS[:, :3]
    assert orc.learned_pool(orc.sum_scores(small), _LEARNED[:3], half=4).tolist() == \
        [A, B, Cc, -1, -1, -1, -1, -1]


def test_learned_mix_hand(orc):
    """Coverage worked out by hand over the whole input (n = 8 <= 4096: the stride
    sample is every point). A covers {B, E, G}; B {E, G}; C {E, F, H}; D {E, G}.
    With R = 2, m_i = 0, 0, 1, 1, 2: sets {A,B}, {A,B}, {A,C}, {A,C}, {C,D}, covering
    3, 3, 5, 5, 4 points; set 2 is the first maximum, picking A then C."""
    pool = np.array([A, B, Cc, D])
    picked, cover = orc.learned_mix(_PTS, pool, n_reps=2, half=2)
    assert cover.tolist() == [3, 3, 5, 5, 4]
    assert picked.tolist() == [A, Cc]
    # n_reps beyond the half is capped at the half
    picked4, cover4 = orc.learned_mix(_PTS, pool, n_reps=64, half=2)
    assert cover4.tolist() == cover.tolist() and picked4.tolist() == picked.tolist()
    # empty slots are skipped in the picks and cover nothing
    picked_e, cover_e = orc.learned_mix(_PTS, np.array([A, -1, Cc, D]), n_reps=2, half=2)
    assert cover_e.tolist() == [3, 3, 5, 5, 4] and picked_e.tolist() == [A, Cc]
    picked_e, cover_e = orc.learned_mix(_PTS, np.array([A, B, -1, D]), n_reps=2, half=2)
    assert cover_e.tolist() == [3, 3, 3, 3, 2] and picked_e.tolist() == [A, B]


def test_learned_mix_stride_sample(orc):
    """With n > the sample cap the coverage is counted on points floor(s n / M) only:
    recounted by brute force on a random input with a small cap."""
    x = datagen.uniform(1000, 3, 4)
    lsc = np.random.default_rng(5).random(1000)
    pool = orc.learned_pool(orc.sum_scores(x), lsc, half=8)
    M = 97
    picked, cover = orc.learned_mix(x, pool, n_reps=8, half=8, sample_cap=M)
    sample = (np.arange(M) * 1000) // M
    for i in range(5):
        mi = i * 8 // 4
        rows = [v for v in list(pool[:8 - mi]) + list(pool[8:8 + mi]) if v >= 0]
        want = _dominates(x[:, rows], x[:, sample]).any(0).sum() if rows else 0
        assert cover[i] == want
    best = int(np.argmax(cover))
    mb = best * 8 // 4
    assert picked.tolist() == [v for v in pool[:8 - mb] if v >= 0] + [v for v in pool[8:8 + mb] if v >= 0]


def test_learned_reduces_to_sorted(orc):
    """A learned score equal to the float32 sum ranks like the sum, so every learned
    candidate is already a sum candidate: the learned half is empty, the mixes
    are nested prefixes of the sum list, and the first (largest) one is chosen, i.e.
    the Sorted representatives."""
    x = datagen.anticorrelated(5000, 4, 3)
    s = orc.sum_scores(x)
    pool = orc.learned_pool(s, s.astype(np.float64))
    assert (pool[64:] == -1).all()
    assert pool[:64].tolist() == orc.select_reps(s, 64).tolist()
    picked, cover = orc.learned_mix(x, pool, n_reps=64)
    assert picked.tolist() == orc.select_reps(s, 64).tolist()
    assert list(cover) == sorted(cover, reverse=True)
    ids, st = orc.pipeline(x, partitioning="sliced", p=8, reps="learned", learned_scores=s.astype(np.float64))
    ids2, st2 = orc.pipeline(x, partitioning="sliced", p=8, reps="sorted")
    assert np.array_equal(ids, ids2)
    assert st["rep_ids"].tolist() == st2["rep_ids"].tolist()
    assert st["n_after_reps"] == st2["n_after_reps"] and st["local_sizes"].tolist() == st2["local_sizes"].tolist()


@pytest.mark.parametrize("gen", ["anticorrelated", "clustered", "uniform"])
def test_learned_pipeline_exact(orc, gen):
    """Any learned score gives the brute-force skyline (representatives are real
    points); the pipeline's pool and picks are the standalone functions'."""
    x = datagen.generate(gen, 3000, 4, 8)
    lsc = np.random.default_rng(2).random(3000) * (1 + x[0])   # an arbitrary score
    ids, st = orc.pipeline(x, partitioning="sliced", p=4, reps="learned", learned_scores=lsc, threads=2)
    assert np.array_equal(ids, orc.sky_brute(x))
    pool = orc.learned_pool(orc.sum_scores(x), lsc)
    assert st["rep_pool"].tolist() == pool.tolist()
    picked, _ = orc.learned_mix(x, pool, 64)
    assert st["rep_ids"].tolist() == picked.tolist()
    assert st["rep_keep"].tolist() == orc.rep_selfilter(x, picked).tolist()


# ----------------------------------------------------------------- Sorted per partition
def test_sorted_part_reps_hand(orc):
    # sums 0.3, 0.1, 0.2, 0.4, 0.0, 0.5 in partitions 1, 0, 1, 0, 2, 2; K = 4, p = 3:
    # ceil(4/3) = 2 per partition
    s = np.array([0.3, 0.1, 0.2, 0.4, 0.0, 0.5], np.float32)
    part = np.array([1, 0, 1, 0, 2, 2], np.uint32)
    assert orc.sorted_part_reps(s, part, 3, 4).tolist() == [1, 3, 2, 0, 4, 5]
    assert orc.sorted_part_reps(s, part, 3, 3).tolist() == [1, 2, 4]
    # an empty partition contributes nothing; ties by id
    s2 = np.array([0.2, 0.2, 0.1], np.float32)
    assert orc.sorted_part_reps(s2, np.array([0, 0, 0], np.uint32), 2, 4).tolist() == [2, 0]


def test_sorted_part_reps_numpy(orc):
    x = datagen.discrete(4000, 4, 6, 20)
    s = orc.sum_scores(x)
    part = orc.sliced_cells(x, 10, 0)
    got = orc.sorted_part_reps(s, part, 10, 64)
    want = []
    for j in range(10):
        mem = np.flatnonzero(part == j)
        want += mem[np.argsort(s[mem], kind="stable")[:7]].tolist()
    assert got.tolist() == want


@pytest.mark.parametrize("part,p,m", [("sliced", 16, None), ("grid", 8, [2, 2, 2]), ("angular", 4, [2, 2])])
def test_sorted_part_pipeline(orc, part, p, m):
    x = datagen.anticorrelated(2500, 3, 11)
    ids, st = orc.pipeline(x, partitioning=part, p=p, m_per_dim=m, reps="sorted_part", n_reps=32,
                           grid_filter=True, grid_filter_m=2)
    assert np.array_equal(ids, orc.sky_brute(x))
    cells = {"sliced": lambda: orc.sliced_cells(x, p, 0), "grid": lambda: orc.grid_cells(x, m),
             "angular": lambda: orc.angular_cells(x, m)}[part]()
    reps = orc.sorted_part_reps(orc.sum_scores(x), cells, p, 32)
    assert st["rep_ids"].tolist() == reps.tolist() and st["n_reps"] == reps.size
    keep = orc.rep_selfilter(x, reps)
    alive = ~orc.grid_filter(x, 2) & ~_dominates(x[:, reps[keep]], x).any(0)
    assert st["n_after_reps"] == alive.sum()


# ----------------------------------------------------------------- reverse counts
def test_domby_hand(orc):
    by = np.array([A, Cc])
    # A dominates B, E, G; C dominates E, F, H
    assert orc.domby(_PTS, by).tolist() == [0, 1, 0, 0, 2, 1, 1, 1]
    assert orc.domby(_PTS, by, which=[E, D]).tolist() == [2, 0]


def test_domby_is_skyline_complement(orc):
    """Over all points, domby > 0 exactly for the points outside the skyline (Def. 1,
    brute force); the total equals the total of the forward counts (Def. 2)."""
    for x in (datagen.discrete(600, 3, 2, 4), datagen.anticorrelated(600, 4, 3)):
        n = x.shape[1]
        allid = np.arange(n)
        c = orc.domby(x, allid)
        sky = np.zeros(n, bool)
        sky[orc.sky_brute(x)] = True
        assert np.array_equal(c > 0, ~sky)
        assert int(c.sum()) == int(orc.domcount(x, allid.astype(np.uint32)).sum())


# ----------------------------------------------------------------- training targets
def test_mlp_targets_closed_forms(orc):
    # the origin dominates every other point; the all-ones corner dominates nothing
    x = np.concatenate([np.zeros((3, 1)), datagen.uniform(499, 3, 1) * 0.98 + 0.01, np.ones((3, 1))],
                       axis=1).astype(np.float32)
    n = x.shape[1]
    sample = np.arange(1, n - 1)          # everything but the origin and the corner
    y, kept = orc.mlp_targets(x, sample)
    assert kept == sample.size
    # dc(origin) = m, so y = -log1p(n) / log1p(n) = -1; the corner has dc = 0
    assert y[0] == -1.0 and y[-1] == 0.0
    # monotone: a point that dominates another has a count at least as large
    D = _dominates(x, x)
    i, j = np.nonzero(D)
    assert (y[i] <= y[j]).all()


def test_mlp_targets_residual(orc):
    x = datagen.anticorrelated(1500, 3, 6)
    n = x.shape[1]
    sample = np.random.default_rng(0).choice(n, 400, replace=False)
    reps = orc.select_reps(orc.sum_scores(x), 16)
    reps = reps[orc.rep_selfilter(x, reps)]
    y, kept = orc.mlp_targets(x, sample, reps)
    res = sample[~_dominates(x[:, reps], x[:, sample]).any(0)]
    assert kept == res.size
    dc = _dominates(x, x[:, res]).sum(1)
    assert np.allclose(y, -np.log1p(dc * n / sample.size) / np.log1p(n), rtol=0, atol=1e-15)


# ----------------------------------------------------------------- work counters
# Six 2-D points: a=(1,5) b=(2,2) c=(3,1) d=(4,4) e=(5,0.5) f=(0.5,6).
_SIX = np.array([[1, 2, 3, 4, 5, 0.5], [5, 2, 1, 4, 0.5, 6]], np.float32)


def test_counters_single_partition_hand(orc):
    """SFS order by (sum, x, y): b (4), c (4), e (5.5), a (6), f (6.5), d (8).
    Comparisons with the skyline found so far: b 0; c 1 (b does not dominate it);
    e 2; a 3; f 4; d 1 (b dominates it at once): 11."""
    ids, st = orc.pipeline(_SIX, partitioning="none")
    assert ids.tolist() == [0, 1, 2, 4, 5]
    assert st["tests_local"] == 11 and st["tests_merge"] == 0
    assert orc.sky_sfs(_SIX, return_tests=True)[1] == 11


def test_counters_sliced_hand(orc):
    """Sliced p = 2 on x: ranks f, a, b | c, d, e. Local: slice 0 in SFS order b, a, f:
    0 + 1 + 2 = 3; slice 1 c, e, d: 0 + 1 + 1 (c dominates d) = 2. NoSeq: u_1 = {c, e}
    against u_0 = (b, a, f) in SFS order, only over points before the query in that
    order: c (key 4, x 3) meets b (key 4, x 2): 1 test; e (key 5.5) meets b: 1 test; a
    and f come after both: 2 in all. The final round instead runs SFS over u =
    b, c, e, a, f: 0 + 1 + 2 + 3 + 4 = 10."""
    ids, st = orc.pipeline(_SIX, partitioning="sliced", p=2)
    assert ids.tolist() == [0, 1, 2, 4, 5]
    assert st["local_sizes"].tolist() == [3, 2]
    assert st["tests_local"] == 5 and st["tests_merge"] == 2
    ids, st = orc.pipeline(_SIX, partitioning="sliced", p=2, merge="global")
    assert ids.tolist() == [0, 1, 2, 4, 5]
    assert st["tests_local"] == 5 and st["tests_merge"] == 10
    ids, st = orc.pipeline(_SIX, partitioning="sliced", p=2, threads=2)
    assert st["tests_local"] == 5 and st["tests_merge"] == 2


def test_counters_bounds(orc):
    """On any input: each partition's SFS makes at least (|r_i| - 1) and at most
    |r_i| (|r_i| - 1) / 2 comparisons; the NoSeq merge at most the uncut count
    sum_i |u_i| |pd_i|. Thread count leaves every counter unchanged."""
    x = datagen.anticorrelated(4000, 4, 9)
    _, st = orc.pipeline(x, partitioning="sliced", p=8)
    _, st4 = orc.pipeline(x, partitioning="sliced", p=8, threads=4)
    assert (st["tests_local"], st["tests_merge"]) == (st4["tests_local"], st4["tests_merge"])
    kept = st["part_kept"]
    assert (kept - 1).clip(0).sum() <= st["tests_local"] <= (kept * (kept - 1) // 2).sum()
    u = st["local_sizes"]
    assert st["tests_merge"] <= sum(u[i] * u[:i].sum() for i in range(8))
