"""Pins for the oracle's skyline algorithms (O1 brute force, O2 2-D, O3 SFS, O4 BNL).

Each check ties the oracle to something other than itself: three independent
algorithms agreeing, closed forms (all-equal, chain, antichain, d = 1), the
top-1-of-a-monotone-function property (Section 2), invariance under
permutations and exact monotone transforms, the worked example's stated
relations (Example 1), and the average-case skyline size of i.i.d. continuous
data (a closed-form recurrence, not in the paper).
"""
import os

import numpy as np
import pytest

import datagen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cases():
    out = []
    seed = 100
    for d in (1, 2, 3, 4, 6, 8):
        for levels in (2, 3, 10, 1000, 0):
            for n in (0, 1, 7, 64, 300):
                seed += 1
                if levels:
                    x = datagen.discrete(n, d, seed, levels)
                else:
                    x = datagen.anticorrelated(n, d, seed) if d > 1 else datagen.uniform(n, d, seed)
                out.append(pytest.param(x, id=f"d{d}-L{levels}-n{n}"))
    return out


@pytest.mark.parametrize("x", _cases())
def test_algorithms_agree(orc, x):
    a = orc.sky_brute(x)
    assert np.array_equal(a, orc.sky_sfs(x))
    assert np.array_equal(a, orc.sky_bnl(x))
    if x.shape[0] == 2:
        assert np.array_equal(a, orc.sky_2d(x))


def _dominates_any(x, t_idx, s_idx):
    """Vectorised: for each s in s_idx, does any t in t_idx dominate it? (test helper)"""
    T = x[:, t_idx][:, :, None]
    S = x[:, s_idx][:, None, :]
    le = (T <= S).all(axis=0)
    lt = (T < S).any(axis=0)
    return (le & lt).any(axis=0)


@pytest.mark.parametrize("seed", range(6))
def test_invariants(orc, seed):
    """Mutual non-dominance and external stability of the output (Def. 1)."""
    for d, levels in ((3, 4), (5, 0), (2, 0), (4, 2)):
        x = datagen.discrete(400, d, seed, levels) if levels else datagen.anticorrelated(400, d, seed)
        sky = orc.sky_sfs(x)
        rest = np.setdiff1d(np.arange(x.shape[1]), sky)
        assert not _dominates_any(x, sky, sky).any()
        if rest.size:
            assert _dominates_any(x, sky, rest).all()


def test_closed_forms(orc):
    # all-equal input: nothing dominates anything
    x = np.full((4, 50), 0.3, np.float32)
    assert np.array_equal(orc.sky_sfs(x), np.arange(50))
    assert np.array_equal(orc.sky_bnl(x), np.arange(50))
    # chain x_i = (i, i, ...) with duplicates of the minimum at ids 3 and 17
    v = np.arange(40, dtype=np.float32) + 1
    v[3] = 0.0
    v[17] = 0.0
    x = np.tile(v, (3, 1))
    assert np.array_equal(orc.sky_sfs(x), [3, 17])
    assert np.array_equal(orc.sky_brute(x), [3, 17])
    # strict 2-D antichain x + y = 1 (distinct points): everything is in the skyline
    t = np.linspace(0, 1, 33, dtype=np.float32)
    x = np.stack([t, (1 - t).astype(np.float32)])
    assert np.array_equal(orc.sky_2d(x), np.arange(33))
    assert np.array_equal(orc.sky_sfs(x), np.arange(33))
    # d = 1: every copy of the minimum value
    x = np.array([[0.5, 0.2, 0.9, 0.2, 0.2, 0.3]], np.float32)
    assert np.array_equal(orc.sky_sfs(x), [1, 3, 4])
    assert np.array_equal(orc.sky_bnl(x), [1, 3, 4])
    # empty input
    e = np.zeros((3, 0), np.float32)
    assert orc.sky_sfs(e).size == 0 and orc.sky_brute(e).size == 0


def test_duplicates_share_fate(orc):
    """Exact duplicates never dominate each other: all copies in or all out."""
    base = datagen.anticorrelated(200, 4, 9)
    x = np.concatenate([base, base[:, :50], base[:, :50]], axis=1)
    sky = set(orc.sky_sfs(x).tolist())
    for i in range(50):
        fate = {i in sky, (200 + i) in sky, (250 + i) in sky}
        assert len(fate) == 1


def test_top1_of_monotone_functions(orc):
    """Section 2: the unique minimiser of a monotone function is in the skyline
    (lexicographic tie-break makes the minimiser unique and still undominated)."""
    rng = np.random.default_rng(5)
    for seed in range(5):
        x = datagen.discrete(500, 4, seed, 7)
        sky = set(orc.sky_sfs(x).tolist())
        fs = [x.astype(np.float64).sum(0)] + [x[k].astype(np.float64) for k in range(4)]
        fs += [(rng.random(4)[:, None] * x).sum(0) for _ in range(5)]
        for f in fs:
            order = np.lexsort(tuple(x[k] for k in reversed(range(4))) + (f,))
            assert int(order[0]) in sky


def test_permutation_and_monotone_transforms(orc):
    x = datagen.discrete(600, 5, 3, 6)
    sky = orc.sky_sfs(x)
    perm = np.random.default_rng(0).permutation(600)
    sky_p = orc.sky_sfs(x[:, perm])
    assert np.array_equal(np.sort(perm[sky_p]), sky)
    # exact, strictly increasing coordinate maps keep the skyline
    assert np.array_equal(orc.sky_sfs(x * np.float32(4.0)), sky)
    # adding 1 keeps the six levels k/6 distinct and ordered
    assert np.array_equal(orc.sky_sfs(x + np.float32(1.0)), sky)
    # dimension order does not matter
    assert np.array_equal(orc.sky_sfs(x[::-1].copy()), sky)


def test_cars_example(orc):
    """Example 1 (Section 2): relations stated in the text on made-up values."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "cars_example.txt")) if not l.startswith("#")]
    names = [r[0] for r in rows]
    x = np.array([[float(r[1]) for r in rows], [float(r[2]) for r in rows]], np.float32)
    want = [i for i, r in enumerate(rows) if r[3] == "1"]
    for f in (orc.sky_brute, orc.sky_2d, orc.sky_sfs, orc.sky_bnl):
        assert f(x).tolist() == want
    assert names[int(np.argmin(x[0]))] == "C1"
    assert names[int(np.argmin(x[1]))] == "C4"
    assert names[int(np.argmin(x[0] + x[1]))] == "C2"


def _expected_maxima(d, n):
    """E|Sky| for n i.i.d. continuous points in d dims: E_1 = 1, E_d(n) = sum_k E_{d-1}(k)/k."""
    e = np.ones(n)
    for _ in range(d - 1):
        e = np.cumsum(e / np.arange(1, n + 1))
    return e[-1]


def test_average_skyline_size(orc):
    """Average skyline cardinality of uniform data matches the closed-form recurrence."""
    assert abs(_expected_maxima(4, 10_000) - 164.7) < 0.1
    for d, n, reps in ((2, 2000, 60), (3, 2000, 40), (4, 4000, 20)):
        sizes = [orc.sky_sfs(datagen.uniform(n, d, 1000 + s)).size for s in range(reps)]
        mean, se = np.mean(sizes), np.std(sizes) / np.sqrt(reps)
        assert abs(mean - _expected_maxima(d, n)) < 4 * se + 0.5
