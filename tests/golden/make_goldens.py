"""Writes the stored expected skylines of the full-size parity tests.

Some workloads are too large for the oracle to finish inside a GPU test (10M x 8
points, 512 instances of up to 200k points, 5M points). This script runs the CPU
oracle on them once and stores, per skyline, its size and the SHA-256 of its ids
(ascending, int64 little-endian), plus the counts of Algorithm 2 that do not depend
on the GPU's options. It calls only ``oracle`` (the skyline) and ``datagen`` (the
seeded inputs); nothing here comes from the GPU path.

    python tests/golden/make_goldens.py [--only NAME] [--threads T]

The skyline does not depend on the partitioning, the representatives or the merge
(Propositions 1 and 2; representatives prune only dominated points), so one oracle
run per input serves every option set the GPU tests run on it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import datagen  # noqa: E402
import oracle  # noqa: E402


def ids_digest(ids: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(ids, dtype="<i8").tobytes()).hexdigest()


def _c5(threads: int) -> dict:
    """Quantised cluster/anticorrelated mixture, 10M x 8, with the workload's Angular
    partitioning and Grid Filtering; Sorted representatives, NoSeq merge."""
    w = datagen.WORKLOADS["angular_mix_10m_d8"]
    x = datagen.workload("angular_mix_10m_d8")
    opts = dict(w["opts"], reps="sorted", merge="noseq")
    t0 = time.time()
    ids, st = oracle.pipeline(x, threads=threads, **opts)
    return {"name": "angular_mix_10m_d8", "n": int(x.shape[1]), "d": int(x.shape[0]),
            "size_sky": int(ids.size), "sha256": ids_digest(ids), "n_after_grid": st["n_after_grid"],
            "part_sizes": st["part_sizes"].tolist(), "oracle": {k: v for k, v in opts.items()},
            "oracle_s": round(time.time() - t0, 1)}


BIG_LOCAL = dict(gen="anticorrelated", n=5_000_000, d=4, seed=61)


def _big_local(threads: int) -> dict:
    """5M anticorrelated points, d = 4: more points than the register-bounded local
    kernel takes, so the unbounded build of the 8-word records runs."""
    g = BIG_LOCAL
    x = datagen.generate(g["gen"], g["n"], g["d"], g["seed"])
    opts = dict(partitioning="sliced", p=16, reps="sorted", n_reps=64, merge="noseq")
    t0 = time.time()
    ids, st = oracle.pipeline(x, threads=threads, **opts)
    return {"name": "ant_5m_d4", **g, "size_sky": int(ids.size), "sha256": ids_digest(ids),
            "size_u": st["size_u"], "n_after_reps": st["n_after_reps"],
            "local_sizes": st["local_sizes"].tolist(), "oracle": opts, "oracle_s": round(time.time() - t0, 1)}


_XS = None


def _one_instance(i: int):
    x = _XS[i]
    if x.shape[1] == 0:
        return i, 0, ids_digest(np.zeros(0, np.int64))
    ids, _ = oracle.pipeline(x, partitioning="sliced", p=16, reps="sorted", n_reps=64, merge="noseq", threads=1)
    return i, int(ids.size), ids_digest(ids)


def _batch(threads: int) -> dict:
    """The 512 instances of the batched workload (sizes log-uniform in [1k, 200k], d in
    {3..8}, uniform / correlated / anticorrelated), one oracle pipeline per instance."""
    global _XS
    _XS = datagen.batch_instances()
    t0 = time.time()
    order = sorted(range(len(_XS)), key=lambda i: -_XS[i].shape[1])   # largest first
    res = {}
    with mp.get_context("fork").Pool(threads) as pool:
        for i, k, h in pool.imap_unordered(_one_instance, order):
            res[i] = (k, h)
    return {"name": "batch_512", "n_instances": len(_XS), "ns": [int(x.shape[1]) for x in _XS],
            "ds": [int(x.shape[0]) for x in _XS], "size_sky": [res[i][0] for i in range(len(_XS))],
            "sha256": [res[i][1] for i in range(len(_XS))], "oracle_s": round(time.time() - t0, 1)}


def _workload_counts(name: str):
    def job(threads: int) -> dict:
        """A named workload under its own options: the skyline and the oracle's counts of
        Algorithm 2, among them the dominance tests of its local SFS and of its merge (the
        algorithmic work the dominance kernels are measured against)."""
        w = datagen.WORKLOADS[name]
        x = datagen.workload(name)
        t0 = time.time()
        ids, st = oracle.pipeline(x, threads=threads, **w["opts"])
        keep = ("n_after_grid", "n_after_reps", "size_u", "size_sky", "tests", "tests_local", "tests_merge")
        return {"name": name, "n": int(x.shape[1]), "d": int(x.shape[0]), "oracle": w["opts"],
                "size_sky": int(ids.size), "sha256": ids_digest(ids), **{k: st[k] for k in keep},
                "oracle_s": round(time.time() - t0, 1)}
    return job


JOBS = {"angular_mix_10m_d8": _c5, "ant_5m_d4": _big_local, "batch_512": _batch,
        "sliced_ant_1m_d6": _workload_counts("sliced_ant_1m_d6"),
        "grid_uniform_10k_d4": _workload_counts("grid_uniform_10k_d4")}


def path(name: str) -> str:
    return os.path.join(HERE, f"sky_{name}.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    oracle.build(force=False)
    for name, fn in JOBS.items():
        if a.only and name != a.only:
            continue
        rec = fn(a.threads)
        with open(path(name), "w") as f:
            json.dump(rec, f, indent=0)
            f.write("\n")
        print(name, {k: v for k, v in rec.items() if k in ("size_sky", "oracle_s")} if name != "batch_512"
              else rec["oracle_s"], flush=True)


if __name__ == "__main__":
    main()
