"""CPU oracle for the partitioned skyline method -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct implementation in C (``skyline_oracle.c``)
with this thin numpy/ctypes wrapper. Only the tests, the package's smoke check
and the benchmark's CPU-baseline leg may import it; the GPU library never does.
It shares no code with the GPU path.

Functions (all take float32 SoA points of shape (d, N)):

* ``sky_brute``   -- O1, the skyline definition (Def. 1) by brute force.
* ``sky_2d``      -- O2, exact 2-D skyline by sort and scan.
* ``sky_sfs``     -- O3, SFS (Algorithm 1) with a lexicographic float64-sum key.
* ``sky_bnl``     -- O4, block nested loops with an unbounded window.
* ``pipeline``    -- O5/O6, Algorithm 2 with Grid / Angular / Sliced partitioning,
  Grid Filtering, representative filtering and the NoSeq or sequential merge;
  ``threads > 1`` runs the per-partition phases on host threads.
* ``grid_cells``, ``angular_cells``, ``sliced_cells``, ``grid_filter``,
  ``sum_scores``, ``select_reps``, ``rep_selfilter`` -- the pipeline's steps.
* ``domcount``    -- O8, dominance counts against a sample (Def. 2); ``domby`` the
  reverse count (how many of a set dominate each point).
* ``learned_pool``, ``learned_mix`` -- the learned representatives' candidate pool
  and the coverage choice among its mixes; ``sorted_part_reps`` -- Sorted
  representatives taken per partition (Section 4.1).
* ``mlp_targets`` -- the scorer's training targets from dominance counts.
* ``mlp_*``       -- O7, the monotone MLP scorer in float64 (forward, loss and
  gradient, Adam step with projection onto non-negative weights).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "skyline_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PART = {"none": 0, "grid": 1, "angular": 2, "sliced": 3, "random": 4}
REPS = {"none": 0, "sorted": 1, "scores": 2, "region": 3, "random": 4, "sorted_part": 5, "learned": 6}
POOL_HALF = 64       # learned representatives: candidates per pool half
COVER_SAMPLE = 4096  # learned representatives: stride sample of the coverage count
MERGE = {"noseq": 0, "global": 1}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-pthread", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Opts(C.Structure):
    _fields_ = [("partitioning", C.c_int32), ("p", C.c_int32), ("m_per_dim", C.c_int32 * 16),
                ("slice_dim", C.c_int32), ("reps", C.c_int32), ("n_reps", C.c_int32),
                ("grid_filter", C.c_int32), ("grid_filter_m", C.c_int32),
                ("merge", C.c_int32), ("threads", C.c_int32), ("seed", C.c_uint64),
                ("learned", C.c_void_p)]


class _Stats(C.Structure):
    _fields_ = [("n_in", C.c_int64), ("n_after_grid", C.c_int64), ("n_reps_kept", C.c_int64),
                ("n_after_reps", C.c_int64), ("size_u", C.c_int64), ("size_sky", C.c_int64),
                ("tests", C.c_int64), ("tests_local", C.c_int64), ("tests_merge", C.c_int64),
                ("n_reps", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i64, i32 = C.c_int64, C.c_int32
        for name, res, args in [
            ("or_sky_brute", i64, [P, i64, i32, P]),
            ("or_sky_2d", i64, [P, i64, P]),
            ("or_sky_sfs", i64, [P, i64, i32, P, P]),
            ("or_sky_bnl", i64, [P, i64, i32, P]),
            ("or_grid_cells", i32, [P, i64, i32, P, P]),
            ("or_angular_cells", i32, [P, i64, i32, P, P]),
            ("or_sliced_cells", i32, [P, i64, i32, i32, i32, P]),
            ("or_grid_filter", i64, [P, i64, i32, P, P]),
            ("or_sum_scores", None, [P, i64, i32, P]),
            ("or_region_scores", i32, [P, i64, i32, P]),
            ("or_splitmix64", C.c_uint64, [C.c_uint64, C.c_uint64]),
            ("or_random_scores", None, [i64, C.c_uint64, P]),
            ("or_random_cells", i32, [i64, i32, C.c_uint64, P]),
            ("or_select_reps", i64, [P, i64, i32, P]),
            ("or_rep_selfilter", i64, [P, i64, i32, P, i64, P]),
            ("or_domcount", None, [P, i64, i32, P, i64, P, i64, P]),
            ("or_domby", None, [P, i64, i32, P, i64, P, i64, P]),
            ("or_mlp_targets", i64, [P, i64, i32, P, i64, P, i64, P]),
            ("or_learned_pool", None, [P, P, i64, i32, P]),
            ("or_learned_mix", i64, [P, i64, i32, P, i32, i32, i64, P, P]),
            ("or_sorted_part_reps", i64, [P, i64, P, i32, i32, P]),
            ("or_pipeline", i64, [P, i64, i32, P, P, P, P, P, P, P, P, P, P]),
            ("or_mlp_nparams", i64, [i32, i32]),
            ("or_mlp_forward", None, [P, i32, i32, P, i64, i32, P, P]),
            ("or_mlp_loss_grad", C.c_double, [P, i32, i32, P, i64, P, i32, P]),
            ("or_mlp_adam", None, [P, P, P, P, i32, i32, C.c_double, C.c_double, C.c_double,
                                   C.c_double, i64]),
        ]:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _pts(pts) -> np.ndarray:
    a = np.ascontiguousarray(pts, dtype=np.float32)
    if a.ndim != 2:
        raise ValueError("points must be (d, N)")
    return a


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _ids(flags: np.ndarray) -> np.ndarray:
    return np.flatnonzero(flags).astype(np.int64)


def sky_brute(pts) -> np.ndarray:
    a = _pts(pts)
    d, n = a.shape
    f = np.zeros(n, np.uint8)
    lib().or_sky_brute(_p(a), n, d, _p(f))
    return _ids(f)


def sky_2d(pts) -> np.ndarray:
    a = _pts(pts)
    if a.shape[0] != 2:
        raise ValueError("sky_2d needs d == 2")
    f = np.zeros(a.shape[1], np.uint8)
    lib().or_sky_2d(_p(a), a.shape[1], _p(f))
    return _ids(f)


def sky_sfs(pts, return_tests: bool = False):
    a = _pts(pts)
    d, n = a.shape
    f = np.zeros(n, np.uint8)
    t = np.zeros(1, np.int64)
    lib().or_sky_sfs(_p(a), n, d, _p(f), _p(t))
    return (_ids(f), int(t[0])) if return_tests else _ids(f)


def sky_bnl(pts) -> np.ndarray:
    a = _pts(pts)
    d, n = a.shape
    f = np.zeros(n, np.uint8)
    lib().or_sky_bnl(_p(a), n, d, _p(f))
    return _ids(f)


def _check(rc: int, what: str):
    if rc == -3:
        raise ValueError(f"{what}: coordinates outside [0,1]")
    if rc < 0:
        raise ValueError(f"{what}: invalid arguments (rc={rc})")


def grid_cells(pts, m) -> np.ndarray:
    a = _pts(pts)
    d, n = a.shape
    mm = np.ascontiguousarray(np.broadcast_to(np.asarray(m, np.int32), (d,)))
    out = np.zeros(n, np.uint32)
    _check(lib().or_grid_cells(_p(a), n, d, _p(mm), _p(out)), "grid_cells")
    return out


def angular_cells(pts, m) -> np.ndarray:
    a = _pts(pts)
    d, n = a.shape
    mm = np.ascontiguousarray(np.broadcast_to(np.asarray(m, np.int32), (max(d - 1, 1),)))
    out = np.zeros(n, np.uint32)
    _check(lib().or_angular_cells(_p(a), n, d, _p(mm), _p(out)), "angular_cells")
    return out


def sliced_cells(pts, p: int, slice_dim: int = 0) -> np.ndarray:
    a = _pts(pts)
    d, n = a.shape
    out = np.zeros(n, np.uint32)
    _check(lib().or_sliced_cells(_p(a), n, d, slice_dim, p, _p(out)), "sliced_cells")
    return out


def grid_filter(pts, m) -> np.ndarray:
    """Boolean mask of points discarded by Grid Filtering."""
    a = _pts(pts)
    d, n = a.shape
    mm = np.ascontiguousarray(np.broadcast_to(np.asarray(m, np.int32), (d,)))
    out = np.zeros(n, np.uint8)
    _check(lib().or_grid_filter(_p(a), n, d, _p(mm), _p(out)), "grid_filter")
    return out.astype(bool)


def sum_scores(pts) -> np.ndarray:
    a = _pts(pts)
    d, n = a.shape
    out = np.zeros(n, np.float32)
    lib().or_sum_scores(_p(a), n, d, _p(out))
    return out


def region_scores(pts) -> np.ndarray:
    """-V(DR(t)) = -prod (1 - t[i]) in float32 (Region representatives, Section 4.1)."""
    a = _pts(pts)
    d, n = a.shape
    out = np.zeros(n, np.float32)
    _check(lib().or_region_scores(_p(a), n, d, _p(out)), "region_scores")
    return out


def splitmix64(seed: int, i: int) -> int:
    """Draw i (0-based) of SplitMix64 from state `seed`."""
    return int(lib().or_splitmix64(seed & (2**64 - 1), i))


def random_scores(n: int, seed: int) -> np.ndarray:
    out = np.zeros(n, np.float32)
    lib().or_random_scores(n, seed & (2**64 - 1), _p(out))
    return out


def random_cells(n: int, p: int, seed: int) -> np.ndarray:
    out = np.zeros(max(n, 1), np.uint32)
    _check(lib().or_random_cells(n, p, seed & (2**64 - 1), _p(out)), "random_cells")
    return out[:n]


def select_reps(score, k: int) -> np.ndarray:
    s = np.ascontiguousarray(score, np.float32)
    ids = np.zeros(max(k, 1), np.int64)
    c = lib().or_select_reps(_p(s), s.size, k, _p(ids))
    return ids[:c]


def rep_selfilter(pts, ids) -> np.ndarray:
    a = _pts(pts)
    d, n = a.shape
    ids = np.ascontiguousarray(ids, np.int64)
    keep = np.zeros(max(ids.size, 1), np.uint8)
    lib().or_rep_selfilter(_p(a), n, d, _p(ids), ids.size, _p(keep))
    return keep[:ids.size].astype(bool)


def domcount(pts, sample, which=None) -> np.ndarray:
    a = _pts(pts)
    d, n = a.shape
    s = np.ascontiguousarray(sample, np.uint32)
    if which is None:
        out = np.zeros(n, np.uint32)
        lib().or_domcount(_p(a), n, d, _p(s), s.size, None, n, _p(out))
    else:
        w = np.ascontiguousarray(which, np.int64)
        out = np.zeros(w.size, np.uint32)
        lib().or_domcount(_p(a), n, d, _p(s), s.size, _p(w), w.size, _p(out))
    return out


def domby(pts, by, which=None) -> np.ndarray:
    """out[a] = number of points by[j] that dominate point which[a] (every point when None)."""
    a = _pts(pts)
    d, n = a.shape
    b = np.ascontiguousarray(by, np.int64)
    if which is None:
        out = np.zeros(n, np.uint32)
        lib().or_domby(_p(a), n, d, _p(b), b.size, None, n, _p(out))
    else:
        w = np.ascontiguousarray(which, np.int64)
        out = np.zeros(w.size, np.uint32)
        lib().or_domby(_p(a), n, d, _p(b), b.size, _p(w), w.size, _p(out))
    return out


def mlp_targets(pts, sample, reps=()):
    """Training targets y (float64, one per point) from dominance counts against the sample
    points that no point of ``reps`` dominates; returns (y, size of that residual sample)."""
    a = _pts(pts)
    d, n = a.shape
    s = np.ascontiguousarray(sample, np.int64)
    r = np.ascontiguousarray(reps, np.int64)
    y = np.zeros(max(n, 1), np.float64)
    kept = lib().or_mlp_targets(_p(a), n, d, _p(s), s.size, _p(r) if r.size else None, r.size, _p(y))
    return y[:n], int(kept)


def learned_pool(sum_score, learned_score, half: int = POOL_HALF) -> np.ndarray:
    """Slots [0, half): the half smallest by (sum, id); [half, 2 half): the half smallest by
    (learned score, id), -1 where already a sum candidate or past n."""
    s = np.ascontiguousarray(sum_score, np.float32)
    g = np.ascontiguousarray(learned_score, np.float64)
    if s.size != g.size:
        raise ValueError("one sum and one learned score per point")
    pool = np.zeros(2 * half, np.int64)
    lib().or_learned_pool(_p(s), _p(g), s.size, half, _p(pool))
    return pool


def learned_mix(pts, pool, n_reps: int = 64, half: int = POOL_HALF, sample_cap: int = COVER_SAMPLE):
    """The mix of the pool's halves that covers the most of the stride sample: (picked ids,
    the five coverage counts)."""
    a = _pts(pts)
    d, n = a.shape
    pl = np.ascontiguousarray(pool, np.int64)
    if pl.size != 2 * half:
        raise ValueError("pool must hold 2 * half slots")
    picked = np.zeros(max(2 * half, 1), np.int64)
    cover = np.zeros(5, np.int64)
    c = lib().or_learned_mix(_p(a), n, d, _p(pl), half, n_reps, sample_cap, _p(picked), _p(cover))
    return picked[:c], cover


def sorted_part_reps(sum_score, part, p: int, k: int) -> np.ndarray:
    """Sorted representatives per partition: the ceil(k / p) smallest by (sum, id) of each."""
    s = np.ascontiguousarray(sum_score, np.float32)
    pt = np.ascontiguousarray(part, np.uint32)
    ids = np.zeros(max(k + p, 1), np.int64)
    c = lib().or_sorted_part_reps(_p(s), s.size, _p(pt), p, k, _p(ids))
    return ids[:c]


def pipeline(pts, partitioning: str = "sliced", p: int = 16, m_per_dim=None, slice_dim: int = 0,
             reps: str = "none", n_reps: int = 64, scores=None, learned_scores=None,
             grid_filter: bool = False, grid_filter_m: int = 0, merge: str = "noseq", threads: int = 1,
             seed: int = 0, **_ignored):
    """Algorithm 2 with the paper's options. Returns (ids, stats dict).

    ``reps``: "sorted" (global), "sorted_part" (per partition), "region", "random",
    "scores" (the n_reps smallest of ``scores``, float32) or "learned" (the pool and mix
    rule over ``learned_scores``, float64, one per point)."""
    a = _pts(pts)
    d, n = a.shape
    o = _Opts()
    o.partitioning = PART[partitioning]
    o.p = 1 if partitioning == "none" else int(p)
    if m_per_dim is not None:
        for k, v in enumerate(m_per_dim):
            o.m_per_dim[k] = int(v)
    o.slice_dim = slice_dim
    o.reps = REPS[reps]
    o.n_reps = n_reps if reps != "none" else 0
    o.grid_filter = int(bool(grid_filter))
    o.grid_filter_m = int(grid_filter_m)
    o.merge = MERGE[merge]
    o.threads = int(threads)
    o.seed = int(seed) & (2**64 - 1)
    np_ = o.p
    st = _Stats()
    f = np.zeros(n, np.uint8)
    psz = np.zeros(np_, np.int64)
    pkept = np.zeros(np_, np.int64)
    lsz = np.zeros(np_, np.int64)
    rid = np.full(max(n_reps + np_, 1), -1, np.int64)
    rkeep = np.zeros(max(n_reps + np_, 1), np.uint8)
    pool = np.full(2 * POOL_HALF, -1, np.int64)
    sc = None
    if o.reps == REPS["scores"]:
        if scores is None:
            raise ValueError("reps='scores' needs scores")
        sc = np.ascontiguousarray(scores, np.float32)
    lsc = None
    if o.reps == REPS["learned"]:
        if learned_scores is None:
            raise ValueError("reps='learned' needs learned_scores")
        lsc = np.ascontiguousarray(learned_scores, np.float64)
        if lsc.size != n:
            raise ValueError("one learned score per point")
        o.learned = lsc.ctypes.data
    rc = lib().or_pipeline(_p(a), n, d, C.byref(o), _p(sc) if sc is not None else None, _p(f),
                           C.byref(st), _p(psz), _p(pkept), _p(lsz), _p(rid), _p(rkeep), _p(pool))
    _check(rc, "pipeline")
    stats = {k: int(getattr(st, k)) for k, _ in _Stats._fields_}
    stats["part_sizes"] = psz
    stats["part_kept"] = pkept
    stats["local_sizes"] = lsz
    if o.reps:
        k = stats["n_reps"]
        stats["rep_ids"] = rid[:k]
        stats["rep_keep"] = rkeep[:k].astype(bool)
    if o.reps == REPS["learned"]:
        stats["rep_pool"] = pool
    return _ids(f), stats


# ---------------------------------------------------------------- MLP (O7)
def mlp_nparams(d: int, h: int) -> int:
    return int(lib().or_mlp_nparams(d, h))


def mlp_forward(params, d: int, h: int, pts, round_mode: int = 1, return_acts: bool = False):
    """Scores g (float64); with return_acts also the pre-activations z1, z2 as (N, h) arrays."""
    P = np.ascontiguousarray(params, np.float64)
    a = _pts(pts)
    n = a.shape[1]
    g = np.zeros(n, np.float64)
    acts = np.zeros((n, 2 * h), np.float64) if return_acts else None
    lib().or_mlp_forward(_p(P), d, h, _p(a), n, round_mode, _p(g), _p(acts) if return_acts else None)
    return (g, acts[:, :h], acts[:, h:]) if return_acts else g


def mlp_loss_grad(params, d: int, h: int, pts, y, round_mode: int = 1):
    P = np.ascontiguousarray(params, np.float64)
    a = _pts(pts)
    yy = np.ascontiguousarray(y, np.float64)
    g = np.zeros(P.size, np.float64)
    loss = lib().or_mlp_loss_grad(_p(P), d, h, _p(a), a.shape[1], _p(yy), round_mode, _p(g))
    return float(loss), g


def mlp_adam(params, m, v, grad, d: int, h: int, lr: float, t: int,
             beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """In place on float64 arrays params, m, v."""
    lib().or_mlp_adam(_p(params), _p(m), _p(v), _p(np.ascontiguousarray(grad, np.float64)), d, h,
                      lr, beta1, beta2, eps, t)
