#!/usr/bin/env python3
"""Benchmark of the partitioned exact skyline on one MI355X.

Workload (default): 1,000,000 anticorrelated points, d = 6, Sliced partitioning
p = 16 on dimension 0, 64 Sorted representatives, NoSeq merge. A step is one
blocking skyline call (every step of the path: ingest, representatives,
filters, partitioning, presort, local skylines, merge, ascending ids copied to
host memory) with the input already resident in HBM.

Prints one JSON line: throughput in input Mpoints/s, the roofline of the
dominant kernel (timed live with HIP events on the call's stream), the CPU
oracle timed on the host cores, and, unless --no-learned, the learned-versus-
Sorted representative comparison on fresh inputs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "input Mpoints/s to exact skyline (d=6 anticorr); learned vs sorted reps speedup"
# Dense peak of 32-bit VALU lane operations: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


SHIPPED_TUNING = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2411_14968_amd", "tuning",
                              "gfx950_256cu.txt")


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sliced_ant_1m_d6")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the 10k x 4 Grid and 10M x 8 Angular legs")
    ap.add_argument("--no-tune", action="store_true", help="use the built-in work splits instead of autotuning")
    ap.add_argument("--tune-file", default=SHIPPED_TUNING,
                    help="tuning table to load (no search) when it exists and was tuned on this device; "
                         "otherwise the bench autotunes and writes the table there")
    ap.add_argument("--retune", action="store_true", help="autotune even when the tuning table loads")
    ap.add_argument("--experiments", default="",
                    help="instead of the benchmark line: write the paper-shaped experiments (representative "
                         "pruning table, N / d / p sweeps on anticorrelated data) as JSON to this file")
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle threads (0 = all host cores, max 16)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size reference dispatch "
                         "for hardware byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path would shard by partitions across GPUs; no multi-GPU path is implemented)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import datagen
    import paper_2411_14968_amd as sky

    if args.experiments:
        experiments(args, sky, datagen, torch, np)
        return
    w = datagen.WORKLOADS[args.workload]
    opts = dict(w["opts"])
    if opts.get("reps") == "learned" or opts.get("presort") == "learned":
        raise SystemExit("the timed workload uses Sorted representatives; learned runs are the comparison leg")
    n, d = w["n"], w["d"]
    x = datagen.workload(args.workload)
    pts = torch.from_numpy(x).cuda()
    ctx = sky.context()
    out = torch.empty(n, dtype=torch.int64).pin_memory()
    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(**extra):
        return sky.skyline(pts, ctx=ctx, out=out, **opts, **extra)

    # work splits of the dominance kernels for this (d, n), picked before the timed region
    tuning = {"params": sky.tune_default(d), "source": "built-in"}
    loaded = False
    if not args.no_tune and not args.retune and args.tune_file and os.path.exists(args.tune_file):
        try:
            sky.tune_load(args.tune_file, ctx=ctx)
            loaded = True
        except sky.SkylineError as e:   # tuned on another device
            print(f"tuning table not used: {e}", file=sys.stderr)
    if loaded:
        tuning = {"params": sky.tune_get(d, n, ctx=ctx)[0], "source": f"loaded {os.path.relpath(args.tune_file)}"}
    elif not args.no_tune:
        t = sky.autotune(pts, trials=5, ctx=ctx, **opts)
        tuning = {"params": t["params"], "source": "autotuned", "median_ms_builtin": round(t["base_ms"], 4),
                  "median_ms_tuned": round(t["best_ms"], 4)}

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ids = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n / (ms_per_step * 1e-3) / 1e6
    gpu_ids = ids.numpy().copy()

    # per-step device times from HIP events recorded on the call's stream
    phases = None
    for _ in range(args.steps):
        _, st = sky.skyline(pts, ctx=ctx, out=out, return_stats=True, phase_times=True, **opts)
        ph = st["ms_phase"]
        phases = ph if phases is None else {k: phases[k] + ph[k] for k in ph}
    phases = {k: v / args.steps for k, v in phases.items()}
    stats = {k: v for k, v in st.items() if k in ("n_after_reps", "size_u", "size_sky", "n_reps_kept")}
    # one instrumented call: the lane tests the dominance kernels issue (same result)
    ids_w, st_w = sky.skyline(pts, ctx=ctx, out=out, return_stats=True, count_work=True, **opts)
    work = st_w["work"]
    assert np.array_equal(ids_w.numpy(), gpu_ids)

    rec = {"metric": METRIC, "value": round(value, 3), "unit": "Mpoints/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
           "data": "synthetic",
           "config": {"workload": args.workload, "n": n, "d": d, "generator": w["gen"], "seed": w["seed"],
                      **{k: v for k, v in opts.items()}},
           "phase_ms": {k: round(v, 4) for k, v in phases.items()}, "counts": stats, "tuning": tuning}

    # Roofline of the dominance kernels (VALU compare-bound): the algorithmic work is the
    # oracle's dominance-test count for the same call (its local SFS and its merge, same
    # options), d compares per test, over the kernel's device time (HIP events on the
    # call's stream). The kernels skip whole blocks of the scan by their lower corners,
    # so they can perform fewer tests than the sequential scan counts; the tests they did
    # perform (instrumented call) are reported beside it.
    oc = oracle_counts(args.workload, x, opts, args)
    kern = {}
    for key, kname, ph in (("local", "k_local_items", "local_kernel"), ("merge", "k_merge_items", "merge_kernel")):
        t = phases[ph]
        w_alg = oc[f"tests_{key}"]
        perf = work[f"{key}_alive_tests"] + work[f"{key}_corner_checks"]
        kern[key] = {"kernel": kname, "kernel_ms": round(t, 4), "w_alg_tests": w_alg,
                     "achieved_TOPs": round(w_alg * d / (t * 1e-3) / 1e12, 4),
                     "frac": round(w_alg * d / (t * 1e-3) / 1e12 / VALU_PEAK_TOPS, 4),
                     "performed_tests": work[f"{key}_alive_tests"], "corner_checks": work[f"{key}_corner_checks"],
                     "issued_lane_tests": work[f"{key}_tests"],
                     "performed_frac": round(perf * d / (t * 1e-3) / 1e12 / VALU_PEAK_TOPS, 4),
                     "traffic": traffic_for(kname, args.workload, tuning["params"])}
    dom = max(kern, key=lambda k: kern[k]["kernel_ms"])
    kd = kern[dom]
    rec["roofline"] = {"bound": "alu", "kernel": kd["kernel"], "achieved": kd["achieved_TOPs"],
                       "peak": round(VALU_PEAK_TOPS, 4), "unit": "TOP/s", "frac": kd["frac"],
                       "traffic": kd["traffic"],
                       "work": f"{kd['w_alg_tests']} dominance tests (the oracle's {dom} count for the same call) "
                               f"x d={d} compares, over the kernel's device time",
                       "kernel_ms": kd["kernel_ms"], "kernels": kern}
    rec["work"] = work
    rec["hbm"] = stream_phases(n, d, phases, oc, args.workload)
    if not args.no_cpu_baseline:
        import oracle
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        c0 = time.perf_counter()
        oids, ost = oracle.pipeline(x, threads=threads, **opts)
        c1 = time.perf_counter()
        rec["cpu_baseline"] = {"value": round(n / (c1 - c0) / 1e6, 4), "unit": "Mpoints/s", "cores": threads,
                               "kind": "oracle", "sample": f"the full {n} x {d} input, one pipeline call "
                                                            f"({c1 - c0:.2f} s)"}
        rec["exact"] = bool(np.array_equal(oids, gpu_ids))
        assert ost["tests_local"] == oc["tests_local"] and ost["tests_merge"] == oc["tests_merge"]
    else:
        rec["exact"] = bool(len(gpu_ids) == oc["size_sky"] and ids_digest(gpu_ids) == oc["sha256"])
    if not args.no_configs:
        rec["configs"] = {"C1": c1_leg(sky, datagen, torch, np, ctx), "C5": c5_leg(sky, datagen, torch, np, ctx)}
    if not args.no_learned:
        rec["learned"] = learned_leg(sky, datagen, torch, np, ctx)
    if not args.no_batch:
        rec["batch"] = batch_leg(sky, datagen, torch, np, ctx, tune=not args.no_tune and not loaded)
    if args.tune_file and tuning["source"] == "autotuned" and args.tune_file != SHIPPED_TUNING:
        sky.tune_save(args.tune_file, ctx=ctx)
    print(json.dumps(rec), flush=True)


def experiments(args, sky, datagen, torch, np):
    """Synthetic stand-ins for the paper's experiments (Section 5), input resident in HBM:
    - the pruning of the representative strategies (Fig. 3: uniform, correlated,
      anticorrelated and clustered data, d = 4): Sorted, Region, random, Sorted per
      partition and learned representatives;
    - NoSeq versus the sequential final round on the same partitioning (Prop. 2, Section 4.2);
    - the sweeps of Table 1 over the dataset size N, the dimensions d and the partitions p
      on anticorrelated data (defaults N = 1M, d = 4, p = 120);
    - inputs shaped like the paper's two real datasets (Section 5; stand-ins, see datagen).
    Each timed point is the median of 3 calls after one warm-up call. Every point the CPU
    oracle finishes (inputs up to about 3.6M points) is checked against the oracle's skyline
    of its input. The cores axis of Table 1 has no counterpart on one GPU."""
    import oracle
    from paper_2411_14968_amd.learned import train_scorer
    ctx = sky.context()
    if os.path.exists(SHIPPED_TUNING):
        try:
            sky.tune_load(SHIPPED_TUNING, ctx=ctx)
        except sky.SkylineError:
            pass
    threads = args.cpu_threads or min(16, os.cpu_count() or 1)
    res = {"device": torch.cuda.get_device_name(0), "pruning": [], "merge": [], "sweeps": [], "real_shaped": []}

    def log(row):
        print(json.dumps(row), file=sys.stderr, flush=True)

    def truth(x):
        """The oracle's skyline of x (it does not depend on the options: Props. 1 and 2)."""
        ids, _ = oracle.pipeline(x, partitioning="sliced", p=16, reps="sorted", n_reps=64, threads=threads)
        return ids

    def timed(pts, **opts):
        n = pts.shape[1]
        out = torch.empty(n, dtype=torch.int64).pin_memory()
        ids = sky.skyline(pts, ctx=ctx, out=out, **opts)
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ids = sky.skyline(pts, ctx=ctx, out=out, **opts)
            ts.append((time.perf_counter() - t0) * 1e3)
        got = ids.numpy().copy()
        _, st = sky.skyline(pts, ctx=ctx, return_stats=True, **opts)
        return sorted(ts)[1], got, st

    # Fig. 3: fraction of the input discarded by 64 representatives
    t0 = time.perf_counter()
    train = [torch.from_numpy(datagen.generate(g, 1_000_000, 4, s)).cuda() for g, s in datagen.TRAIN_SETS]
    scorer, _ = train_scorer(train, epochs=2, batch=4096, lr=2e-3)
    del train
    res["scorer_d4_train_s"] = round(time.perf_counter() - t0, 2)
    for gen in ("uniform", "correlated", "anticorrelated", "clustered"):
        x = torch.from_numpy(datagen.generate(gen, 1_000_000, 4, 7)).cuda()
        row = {"data": gen, "n": 1_000_000, "d": 4}
        for reps, part in (("sorted", "none"), ("region", "none"), ("random", "none"), ("sorted_part", "sliced"),
                           ("learned", "none")):
            _, st = sky.skyline(x, ctx=ctx, return_stats=True, partitioning=part, p=16, reps=reps, n_reps=64, seed=1,
                                model=scorer if reps == "learned" else None)
            row[reps] = round(1.0 - st["n_after_reps"] / st["n_in"], 4)
        res["pruning"].append(row)
        log(row)
    scorer.close()

    # NoSeq versus the final SFS round, same partitioning and representatives
    for label, gen, n, d, opts in (
            ("C2", "anticorrelated", 1_000_000, 6, dict(partitioning="sliced", p=16, reps="sorted", n_reps=64)),
            ("defaults", "anticorrelated", 1_000_000, 4, dict(partitioning="sliced", p=120, reps="sorted", n_reps=64)),
            ("defaults", "anticorrelated", 1_000_000, 4,
             dict(partitioning="angular", p=125, m_per_dim=[5, 5, 5], reps="sorted", n_reps=64))):
        xh = datagen.generate(gen, n, d, 2 if label == "C2" else 9)
        want = truth(xh)
        x = torch.from_numpy(xh).cuda()
        for merge in ("noseq", "global"):
            ms, got, st = timed(x, merge=merge, **opts)
            row = {"case": label, "n": n, "d": d, "partitioning": opts["partitioning"], "p": opts["p"], "merge": merge,
                   "ms": round(ms, 3), "merge_ms_phase": None, "size_u": st["size_u"], "size_sky": len(got),
                   "exact": bool(np.array_equal(got, want))}
            _, stp = sky.skyline(x, ctx=ctx, return_stats=True, phase_times=True, merge=merge, **opts)
            row["merge_ms_phase"] = round(stp["ms_phase"]["merge_kernel"], 4)
            res["merge"].append(row)
            log(row)
        del x

    def strategies(d):
        ma = min(16, max(1, round(120 ** (1.0 / max(d - 1, 1)))))   # slices per angle, p close to 120
        mg = max(1, round(120 ** (1.0 / d)))
        return {"SlicedRep+NoSeq": dict(partitioning="sliced", p=120, reps="sorted", n_reps=64),
                "Sliced+NoSeq": dict(partitioning="sliced", p=120, reps="none"),
                "AngularRep+NoSeq": dict(partitioning="angular", p=ma ** (d - 1), m_per_dim=[ma] * (d - 1),
                                         reps="sorted", n_reps=64),
                "Grid": dict(partitioning="grid", p=mg ** d, m_per_dim=[mg] * d, reps="none", merge="global"),
                "Random": dict(partitioning="random", p=120, reps="none", merge="global", seed=1)}

    def point(axis, value, xh, names, out, **over):
        d, n = xh.shape
        want = truth(xh) if n <= 4_000_000 else None
        x = torch.from_numpy(xh).cuda()
        for name, opts in strategies(d).items():
            if name not in names:
                continue
            opts = dict(opts, **over)
            ms, got, st = timed(x, **opts)
            row = {"axis": axis, "value": value, "n": n, "d": d, "strategy": name, "p": opts["p"],
                   "ms": round(ms, 3), "Mpoints_s": round(n / ms / 1e3, 1), "size_sky": len(got),
                   "size_u": st["size_u"], "n_after_reps": st["n_after_reps"],
                   "exact": None if want is None else bool(np.array_equal(got, want))}
            out.append(row)
            log(row)
        del x
        torch.cuda.empty_cache()

    allnames = ("SlicedRep+NoSeq", "Sliced+NoSeq", "AngularRep+NoSeq", "Grid", "Random")
    for n in (100_000, 500_000, 1_000_000, 5_000_000, 10_000_000, 50_000_000, 100_000_000):
        point("N", n, datagen.generate("anticorrelated", n, 4, 9),
              allnames if n <= 10_000_000 else ("SlicedRep+NoSeq", "AngularRep+NoSeq"), res["sweeps"])
    for d in (2, 3, 5, 6, 7):
        point("d", d, datagen.generate("anticorrelated", 1_000_000, d, 9), ("SlicedRep+NoSeq", "AngularRep+NoSeq"),
              res["sweeps"])
    x4 = datagen.generate("anticorrelated", 1_000_000, 4, 9)
    for p in (60, 240, 360, 600, 1200, 2400, 3600):
        point("p", p, x4, ("SlicedRep+NoSeq", "Sliced+NoSeq", "Random"), res["sweeps"], p=p)
    for name, (gen, n, d, seed) in datagen.REAL_SHAPED.items():
        point("data", name, datagen.generate(gen, n, d, seed), allnames, res["real_shaped"])
    with open(args.experiments, "w") as f:
        json.dump(res, f, indent=1)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden")


def ids_digest(ids) -> str:
    import hashlib
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(ids, dtype="<i8").tobytes()).hexdigest()


def oracle_counts(workload: str, x, opts: dict, args) -> dict:
    """The oracle's skyline digest and counts for this workload: stored by the golden-value
    script (which runs only the oracle) when it holds this workload under the same options,
    else computed here by the oracle."""
    path = os.path.join(GOLDEN, f"sky_{workload}.json")
    if os.path.exists(path):
        with open(path) as f:
            g = json.load(f)
        if g.get("oracle") == opts and "tests_local" in g:
            return g
    import oracle
    ids, st = oracle.pipeline(x, threads=args.cpu_threads or min(16, os.cpu_count() or 1), **opts)
    return {**st, "size_sky": int(ids.size), "sha256": ids_digest(ids)}


def stream_phases(n: int, d: int, phases: dict, oc: dict, workload: str) -> dict:
    """HBM-stream steps: algorithmic bytes (what the step must read and write at least)
    over the step's device time, against 8 TB/s. S = points surviving the filters, U = the
    union of the local skylines, K = the skyline."""
    S, U, K = oc["n_after_reps"], oc["size_u"], oc["size_sky"]
    alg = {"ingest": ((4 * d + 4) * n, "coordinates read, score written"),
           "reps": (4 * n, "scores read once"),
           "filter_partition": ((4 * d + 5) * n, "coordinates read, survivor flag and partition id written"),
           "presort": (5 * n + S * (8 * d + 8), "flags and partition ids read; survivors' coordinates read "
                                                "and written as sorted records with their keys"),
           "union": (S + U * (8 * d + 16), "kill flags read; union records and keys read and written"),
           "output": (n // 8 + 8 * K, "skyline bitmap read, int64 ids written")}
    out = {}
    for ph, (b, what) in alg.items():
        t = phases[ph]
        gbs = b / (t * 1e-3) / 1e9 if t > 0 else 0.0
        out[ph] = {"alg_bytes": b, "ms": round(t, 4), "GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                   "bytes": what}
    prof = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", f"stream_{workload}_hbm.json")
    if os.path.exists(prof):
        with open(prof) as f:
            out["rocprof"] = json.load(f)
    return out


def c1_leg(sky, datagen, torch, np, ctx):
    """Plain method, small: 10,000 uniform points, d = 4, Grid m = 2 (p = 16) with Grid Filtering."""
    import oracle
    name = "grid_uniform_10k_d4"
    w = datagen.WORKLOADS[name]
    x = datagen.workload(name)
    pts = torch.from_numpy(x).cuda()
    out = torch.empty(w["n"], dtype=torch.int64).pin_memory()
    for _ in range(5):
        sky.skyline(pts, ctx=ctx, out=out, **w["opts"])
    ts = []
    for _ in range(50):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ids = sky.skyline(pts, ctx=ctx, out=out, **w["opts"])
        ts.append((time.perf_counter() - t) * 1e3)
    ms = float(np.median(ts))
    want, _ = oracle.pipeline(x, threads=4, **w["opts"])
    return {"workload": name, "ms_per_call": round(ms, 4), "Mpoints_s": round(w["n"] / ms / 1e3, 3),
            "size_sky": int(ids.numel()), "exact": bool(np.array_equal(ids.numpy(), want))}


def c5_leg(sky, datagen, torch, np, ctx):
    """Large with ties: 10M x 8 quantised cluster/anticorrelated mixture, Angular p = 64, Grid
    Filtering m_g = 4, learned representatives from a scorer trained on a fresh 500k mixture
    sample, final SFS round. Exactness against the oracle's stored skyline digest."""
    from paper_2411_14968_amd.learned import train_scorer
    name = "angular_mix_10m_d8"
    w = datagen.WORKLOADS[name]
    t0 = time.perf_counter()
    train = [torch.from_numpy(datagen.mixture_quantized(500_000, 8, 50)).cuda()]
    model, _ = train_scorer(train, epochs=1, batch=4096, lr=2e-3, m=16384)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del train
    x = datagen.workload(name)
    pts = torch.from_numpy(x).cuda()
    out = torch.empty(w["n"], dtype=torch.int64).pin_memory()
    res = {"workload": name, "train_s": round(train_s, 2)}
    with open(os.path.join(GOLDEN, f"sky_{name}.json")) as f:
        g = json.load(f)
    for label, extra in (("learned_reps", {}), ("sorted_reps", {"reps": "sorted"})):
        o = {**w["opts"], **extra}
        for _ in range(2):
            sky.skyline(pts, ctx=ctx, out=out, model=model, **o)
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t = time.perf_counter()
            ids = sky.skyline(pts, ctx=ctx, out=out, model=model, **o)
            ts.append((time.perf_counter() - t) * 1e3)
        ms = float(np.median(ts))
        res[label] = {"ms_per_call": round(ms, 3), "Mpoints_s": round(w["n"] / ms / 1e3, 2),
                      "size_sky": int(ids.numel()),
                      "exact": bool(ids.numel() == g["size_sky"] and ids_digest(ids.numpy()) == g["sha256"])}
    model.close()
    del pts
    torch.cuda.empty_cache()
    return res


def traffic_for(kernel: str, workload: str, splits: dict):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it was
    taken on the current kernel source with the same work splits (else None)."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    h = hashlib.sha256()   # the kernel's source files, in the listed order
    for name in t.get("sources", [t.get("source")]):
        with open(os.path.join(here, "paper_2411_14968_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != t["source_sha256"]:
        return None
    if t.get("splits") != splits:
        return None
    return t["hbm_bytes_per_launch"]


def batch_leg(sky, datagen, torch, np, ctx, tune=True):
    """Many independent instances per call: 512 instances, sizes log-uniform in [1k, 200k],
    d uniform in {3..8}, uniform / correlated / anticorrelated at random; Sliced p=16 and 64
    Sorted representatives per instance. Input resident in HBM; per-instance ids to host."""
    xs = datagen.batch_instances()
    packed, ns, ds = sky.pack_instances([torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in xs])
    total = sum(ns)
    if tune:
        t = sky.autotune_batch(packed, ns, ds, trials=3, ctx=ctx)
        tuning = {"source": "autotuned", "params": t["params"], "median_ms_builtin": round(t["base_ms"], 3),
                  "median_ms_tuned": round(t["best_ms"], 3)}
    else:
        # the splits each launch sequence takes: the context's table entry for the
        # group's record width and total point count, else the built-in ones
        groups = {}
        for n_i, d_i in zip(ns, ds):
            w = ((int(d_i) + 5) // 4) * 4
            g = groups.setdefault(w, [0, 0])   # the group's widest d, its points
            g[0] = max(g[0], int(d_i))
            g[1] += int(n_i)
        tuning = {"source": "table lookup per launch sequence", "groups": {}}
        for w, (d_g, n_g) in sorted(groups.items()):
            params, from_table = sky.tune_get(d_g, n_g, ctx=ctx)
            tuning["groups"][f"record_width_{w}"] = {"points": n_g, "params": params,
                                                     "from": "table" if from_table else "built-in"}
    buf = torch.empty(total, dtype=torch.int64)   # the caller's reused output buffer
    for _ in range(2):
        sky.skyline_batch(packed, ns, ds, ctx=ctx, out=buf)
    torch.cuda.synchronize()
    reps = 5
    t = time.perf_counter()
    for _ in range(reps):
        out, st = sky.skyline_batch(packed, ns, ds, ctx=ctx, return_stats=True, out=buf)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / reps
    return {"workload": "512 instances, N_i log-uniform [1k, 200k], d_i in {3..8}", "n_instances": len(xs),
            "points": total, "ms_per_call": round(ms, 3), "Mpoints_s": round(total / ms / 1e3, 2),
            "device_ms": round(st["ms_total"], 3), "launch_sequences": st["n_groups"],
            "skyline_points": st["size_sky"], "tuning": tuning}


def learned_leg(sky, datagen, torch, np, ctx):
    """Learned versus Sorted representatives on fresh 1M x 6 inputs (training excluded from timing)."""
    from paper_2411_14968_amd.learned import train_scorer
    t0 = time.perf_counter()
    train = [torch.from_numpy(datagen.generate(g, 1_000_000, 6, s)).cuda() for g, s in datagen.TRAIN_SETS]
    model, log = train_scorer(train, epochs=2, batch=4096, lr=2e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del train
    res = {"train_s": round(train_s, 2), "train_loss": [round(v, 5) for v in log["loss"]],
           "train_points": log["train_points"]}
    for name in ("learned_ant_1m_d6", "learned_clustered_1m_d6"):
        w = datagen.WORKLOADS[name]
        p = torch.from_numpy(datagen.workload(name)).cuda()
        base = dict(partitioning="sliced", p=16, n_reps=64, merge="noseq")
        row = {}
        ref = None
        for label, o in (("sorted", dict(reps="sorted")),
                         ("learned", dict(reps="learned", model=model)),
                         ("learned_presort_too", dict(reps="learned", presort="learned", model=model))):
            out = torch.empty(w["n"], dtype=torch.int64).pin_memory()
            for _ in range(2):
                sky.skyline(p, ctx=ctx, out=out, **base, **o)
            torch.cuda.synchronize()
            t = time.perf_counter()
            reps = 10
            for _ in range(reps):   # no stats: the calls replay their captured graphs, as in the timed leg
                sky.skyline(p, ctx=ctx, out=out, **base, **o)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t) * 1e3 / reps
            ids, st = sky.skyline(p, ctx=ctx, return_stats=True, **base, **o)   # counts for the row
            if ref is None:
                ref = ids
            row[label] = {"ms": round(ms, 4), "Mpoints_s": round(w["n"] / ms / 1e3, 2),
                          "pruned_by_reps": round(1 - st["n_after_reps"] / w["n"], 5),
                          "size_u": st["size_u"], "exact_same_ids": bool(torch.equal(ids, ref))}
            if "rep_pool" in st:
                learned_half = set(v for v in st["rep_pool"][len(st["rep_pool"]) // 2:] if v >= 0)
                row[label]["picks_from_learned_half"] = sum(1 for r in st["rep_ids"] if r in learned_half)
                row[label]["n_picks"] = len(st["rep_ids"])
        row["speedup"] = round(row["sorted"]["ms"] / row["learned"]["ms"], 4)
        res[name] = row
    model.close()
    return res


if __name__ == "__main__":
    main()
