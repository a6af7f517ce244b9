"""Partitioned exact skylines on MI355X (gfx950).

Python binding of ``libskyline.so`` (C-ABI in ``include/skyline.h``): argument
marshalling only. Every step of the skyline path runs in the library's HIP
kernels; PyTorch supplies device memory and the current stream.

    import torch, paper_2411_14968_amd as sky
    pts = torch.rand(6, 1_000_000, device="cuda")          # SoA (d, N) float32
    ids = sky.skyline(pts, partitioning="sliced", p=16, reps="sorted")

The package refuses to load without the built library: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from collections.abc import Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libskyline.so")

SKY_OK = 0
ERRORS = {-1: "invalid argument", -2: "non-finite coordinate", -3: "coordinate outside [0,1]",
          -4: "output capacity", -5: "out of memory", -6: "HIP error", -7: "model", -8: "file",
          -9: "internal check"}
PART = {"none": 0, "grid": 1, "angular": 2, "sliced": 3, "random": 4}
REPS = {"none": 0, "sorted": 1, "learned": 2, "region": 3, "random": 4, "sorted_part": 5}
MERGE = {"noseq": 0, "global": 1}
PRESORT = {"sum": 0, "learned": 1, "zorder": 2, "zorder_sum": 3}
MLP_HIDDEN = 64


class SkylineError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        self.code = code
        super().__init__(f"{ERRORS.get(code, 'error')} ({code}): {msg}")


class SkyOpts(C.Structure):
    _fields_ = [("partitioning", C.c_int32), ("p", C.c_int32), ("m_per_dim", C.c_int32 * 16),
                ("slice_dim", C.c_int32), ("reps", C.c_int32), ("n_reps", C.c_int32),
                ("grid_filter", C.c_int32), ("grid_filter_m", C.c_int32), ("merge", C.c_int32),
                ("presort", C.c_int32), ("model", C.c_void_p), ("flags", C.c_uint32), ("seed", C.c_uint64)]


class SkyStats(C.Structure):
    _fields_ = [("n_in", C.c_int64), ("n_after_grid", C.c_int64), ("n_reps_kept", C.c_int64),
                ("n_after_reps", C.c_int64), ("size_u", C.c_int64), ("size_sky", C.c_int64),
                ("n_parts", C.c_int32), ("reserved", C.c_int32),
                ("part_sizes", C.POINTER(C.c_int64)), ("part_kept", C.POINTER(C.c_int64)),
                ("local_sizes", C.POINTER(C.c_int64)), ("rep_ids", C.POINTER(C.c_int64)),
                ("rep_keep", C.POINTER(C.c_uint8)), ("n_reps", C.c_int32), ("n_pool", C.c_int32),
                ("rep_pool", C.POINTER(C.c_int64)), ("ms_total", C.c_float),
                ("ms_phase", C.c_float * 8), ("work", C.c_int64 * 6), ("tests", C.c_int64)]

PHASES = ["ingest", "reps", "filter_partition", "presort", "local_kernel", "union", "merge_kernel", "output"]
FLAG_PHASE_TIMES = 1
FLAG_COUNT_WORK = 2
FLAG_NO_GRAPH = 4
WORK = ["local_tests", "local_corner_checks", "merge_tests", "merge_corner_checks", "local_alive_tests",
        "merge_alive_tests"]


class SkyBatchStats(C.Structure):
    _fields_ = [("n_total", C.c_int64), ("size_sky", C.c_int64), ("n_groups", C.c_int32), ("ms_total", C.c_float)]


class SkyTuneParams(C.Structure):
    _fields_ = [("local_ppl", C.c_int32), ("local_seg", C.c_int32), ("merge_ppl", C.c_int32),
                ("merge_seg", C.c_int32), ("wg_per_cu", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class SkyTrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float)]


_lib = None


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2411_14968_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        sig = {
            "sky_create": (C.c_int, [C.POINTER(P), i32]),
            "sky_destroy": (None, [P]),
            "sky_last_error": (C.c_char_p, [P]),
            "sky_opts_default": (None, [C.POINTER(SkyOpts)]),
            "sky_skyline": (C.c_int, [P, P, i64, i32, C.POINTER(SkyOpts), P, i64, C.POINTER(i64),
                                      C.POINTER(SkyStats), P]),
            "sky_mlp_nparams": (i64, [i32, i32]),
            "sky_mlp_create": (C.c_int, [P, i32, i32, P, C.c_uint64, C.POINTER(P)]),
            "sky_mlp_destroy": (None, [P]),
            "sky_mlp_get_params": (C.c_int, [P, P, i64]),
            "sky_mlp_save": (C.c_int, [P, C.c_char_p]),
            "sky_mlp_load": (C.c_int, [P, C.c_char_p, C.POINTER(P)]),
            "sky_mlp_score": (C.c_int, [P, P, P, i64, i32, P, P]),
            "sky_mlp_loss_grad": (C.c_int, [P, P, P, i64, i32, P, P, P, P]),
            "sky_mlp_adam_step": (C.c_int, [P, P, P, C.c_float, C.c_float, C.c_float, C.c_float, i64, P]),
            "sky_mlp_train": (C.c_int, [P, P, P, i64, i32, P, C.POINTER(SkyTrainOpts),
                                        C.POINTER(C.c_float), P]),
            "sky_domcount": (C.c_int, [P, P, i64, i32, P, i64, P, P]),
            "sky_domby": (C.c_int, [P, P, i64, i32, P, i64, P, P]),
            "sky_mlp_targets": (C.c_int, [P, P, i64, i32, P, i64, P, i64, P, C.POINTER(i64), P]),
            "sky_mlp_targets_noalloc": (C.c_int, [P, P, i64, i32, P, i64, P, i64, P, P, P]),
            "sky_skyline_batch": (C.c_int, [P, P, P, P, i32, C.POINTER(SkyOpts), P, i64, P,
                                            C.POINTER(SkyBatchStats), P]),
            "sky_tune_default": (None, [i32, C.POINTER(SkyTuneParams)]),
            "sky_tune_set": (C.c_int, [P, i32, i64, C.POINTER(SkyTuneParams)]),
            "sky_tune_get": (C.c_int, [P, i32, i64, C.POINTER(SkyTuneParams)]),
            "sky_tune_clear": (None, [P]),
            "sky_tune_save": (C.c_int, [P, C.c_char_p]),
            "sky_tune_load": (C.c_int, [P, C.c_char_p]),
            "sky_autotune": (C.c_int, [P, P, i64, i32, C.POINTER(SkyOpts), i32, C.POINTER(SkyTuneParams),
                                       C.POINTER(C.c_float), C.POINTER(C.c_float), P]),
            "sky_autotune_batch": (C.c_int, [P, P, P, P, i32, C.POINTER(SkyOpts), i32, C.POINTER(SkyTuneParams),
                                             C.POINTER(C.c_float), C.POINTER(C.c_float), P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_points(points: torch.Tensor):
    if not isinstance(points, torch.Tensor) or points.dim() != 2:
        raise ValueError("points must be a (d, N) tensor")
    if points.dtype != torch.float32 or not points.is_cuda:
        raise ValueError("points must be float32 on a GPU")
    if not points.is_contiguous():
        raise ValueError("points must be contiguous SoA (d, N)")


class Context:
    """A library context on one device (owns the reusable workspace)."""

    def __init__(self, device: int | None = None):
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = C.c_void_p()
        rc = lib().sky_create(C.byref(h), self.device)
        if rc != SKY_OK:
            raise SkylineError(rc, f"sky_create(device={device})")
        self.h = h

    def error(self) -> str:
        m = lib().sky_last_error(self.h)
        return m.decode() if m else ""

    def close(self):
        if getattr(self, "h", None):
            lib().sky_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts: dict[int, Context] = {}


def context(device: int | None = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    if device not in _contexts:
        _contexts[device] = Context(device)
    return _contexts[device]


def make_opts(partitioning="sliced", p=16, m_per_dim=None, slice_dim=0, reps="sorted", n_reps=64,
              grid_filter=False, grid_filter_m=0, merge="noseq", presort="zorder", model=None,
              phase_times=False, count_work=False, graph=True, seed=0) -> SkyOpts:
    o = SkyOpts()
    lib().sky_opts_default(C.byref(o))
    o.partitioning = PART[partitioning]
    o.p = int(p)
    if m_per_dim is not None:
        for k, v in enumerate(m_per_dim):
            o.m_per_dim[k] = int(v)
    o.slice_dim = int(slice_dim)
    o.reps = REPS[reps]
    o.n_reps = int(n_reps)
    o.grid_filter = int(bool(grid_filter))
    o.grid_filter_m = int(grid_filter_m)
    o.merge = MERGE[merge]
    o.presort = PRESORT[presort]
    o.model = model.h if model is not None else None
    o.flags = ((FLAG_PHASE_TIMES if phase_times else 0) | (FLAG_COUNT_WORK if count_work else 0)
               | (0 if graph else FLAG_NO_GRAPH))
    o.seed = int(seed) & (2**64 - 1)
    return o


def _stats_dict(st: SkyStats) -> dict:
    npart = st.n_parts
    out = {k: int(getattr(st, k)) for k in ("n_in", "n_after_grid", "n_reps_kept", "n_after_reps",
                                             "size_u", "size_sky")}
    out["n_parts"] = npart
    out["ms_total"] = float(st.ms_total)
    out["ms_phase"] = {name: float(st.ms_phase[i]) for i, name in enumerate(PHASES)}
    out["work"] = {name: int(st.work[i]) for i, name in enumerate(WORK)}
    out["tests"] = int(st.tests)
    if npart and st.part_sizes:
        out["part_sizes"] = [st.part_sizes[j] for j in range(npart)]
        out["part_kept"] = [st.part_kept[j] for j in range(npart)]
        out["local_sizes"] = [st.local_sizes[j] for j in range(npart)]
    if st.n_reps:
        out["rep_ids"] = [st.rep_ids[j] for j in range(st.n_reps)]
        out["rep_keep"] = [bool(st.rep_keep[j]) for j in range(st.n_reps)]
    if st.n_pool:
        out["rep_pool"] = [st.rep_pool[j] for j in range(st.n_pool)]
    return out


def skyline(points: torch.Tensor, partitioning: str = "sliced", p: int = 16, m_per_dim=None,
            slice_dim: int = 0, reps: str = "sorted", n_reps: int = 64, grid_filter: bool = False,
            grid_filter_m: int = 0, merge: str = "noseq", presort: str = "zorder", model: "Scorer | None" = None,
            return_stats: bool = False, ctx: Context | None = None, out: torch.Tensor | None = None,
            phase_times: bool = False, count_work: bool = False, graph: bool = True, seed: int = 0):
    """Skyline of the (d, N) float32 device points: ascending int64 ids (CPU tensor).

    Minimises every coordinate; duplicates share one fate. ``return_stats`` adds the
    per-step counts of Algorithm 2 (see ``sky_stats`` in ``include/skyline.h``);
    ``phase_times`` and ``count_work`` fill its step times and dominance-kernel work.
    ``graph=False`` launches every kernel instead of replaying the call's captured graph.
    ``out`` may be a pinned or pageable CPU int64 tensor with room for N ids.
    """
    _check_points(points)
    d, n = points.shape
    ctx = ctx or context(points.device.index)
    o = make_opts(partitioning, p, m_per_dim, slice_dim, reps, n_reps, grid_filter, grid_filter_m, merge,
                  presort, model, phase_times, count_work, graph, seed)
    if out is None:
        out = torch.empty(max(n, 1), dtype=torch.int64)
    elif out.dtype != torch.int64 or out.device.type != "cpu" or out.numel() < n:
        raise ValueError("out must be a CPU int64 tensor with room for N ids")
    nout = C.c_int64(0)
    st = SkyStats()
    rc = lib().sky_skyline(ctx.h, C.c_void_p(points.data_ptr()), n, d, C.byref(o),
                           C.c_void_p(out.data_ptr()), out.numel(), C.byref(nout),
                           C.byref(st) if return_stats else None, _stream())
    if rc != SKY_OK:
        raise SkylineError(rc, ctx.error())
    ids = out[:nout.value]
    return (ids, _stats_dict(st)) if return_stats else ids


def pack_instances(instances: list[torch.Tensor]) -> tuple[torch.Tensor, list[int], list[int]]:
    """Concatenate (d_i, N_i) float32 device instances into the packed layout of
    ``sky_skyline_batch``; returns (packed, ns, ds)."""
    for x in instances:
        _check_points(x)
    ns = [int(x.shape[1]) for x in instances]
    ds = [int(x.shape[0]) for x in instances]
    if not instances:
        return torch.empty(0, dtype=torch.float32), ns, ds
    return torch.cat([x.reshape(-1) for x in instances]).contiguous(), ns, ds


class BatchIds(Sequence):
    """Per-instance skyline ids of a batched call: item i is instance i's ascending ids, a view
    of the flat buffer ``flat`` from ``offsets[i]`` to ``offsets[i + 1]`` (views are made on access)."""

    def __init__(self, flat: torch.Tensor, offsets: list[int]):
        self.flat = flat
        self.offsets = offsets

    def __len__(self):
        return len(self.offsets) - 1

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self[j] for j in range(*i.indices(len(self)))]
        n = len(self)
        if i < 0:
            i += n
        if not 0 <= i < n:
            raise IndexError(i)
        return self.flat[self.offsets[i]:self.offsets[i + 1]]


def skyline_batch(packed: torch.Tensor, ns: list[int], ds: list[int], partitioning: str = "sliced", p: int = 16,
                  reps: str = "sorted", n_reps: int = 64, presort: str = "zorder", return_stats: bool = False,
                  ctx: Context | None = None, out: torch.Tensor | None = None):
    """Skylines of many instances (``pack_instances`` layout) in one launch sequence per
    record width: a ``BatchIds`` sequence of ascending int64 id tensors (CPU), one per
    instance, all views of one buffer. ``out`` (a CPU int64 tensor with room for sum(ns) ids) is that buffer when
    given; a caller that reuses it avoids touching fresh memory on every call."""
    if len(ns) != len(ds):
        raise ValueError("ns and ds must have one entry per instance")
    total = sum(n * d for n, d in zip(ns, ds))
    if total and (not packed.is_cuda or packed.dtype != torch.float32 or not packed.is_contiguous()
                  or packed.numel() < total):
        raise ValueError("packed must be a contiguous float32 device tensor holding every instance")
    dev = packed.device.index if packed.is_cuda else torch.cuda.current_device()
    ctx = ctx or context(dev)
    o = make_opts(partitioning, p, None, 0, reps, n_reps, False, 0, "noseq", presort, None)
    n_inst = len(ns)
    ns_a = (C.c_int64 * max(n_inst, 1))(*ns)
    ds_a = (C.c_int32 * max(n_inst, 1))(*ds)
    offs = (C.c_int64 * (n_inst + 1))()
    cap = max(sum(ns), 1)
    if out is None:
        out = torch.empty(cap, dtype=torch.int64)   # filled by host copies: pageable memory is enough
    elif out.dtype != torch.int64 or out.device.type != "cpu" or not out.is_contiguous() or out.numel() < cap:
        raise ValueError("out must be a contiguous CPU int64 tensor with room for sum(ns) ids")
    else:
        cap = out.numel()
    st = SkyBatchStats()
    rc = lib().sky_skyline_batch(ctx.h, C.c_void_p(packed.data_ptr() if total else 0), ns_a, ds_a, n_inst,
                                 C.byref(o), C.c_void_p(out.data_ptr()), cap, offs, C.byref(st), _stream())
    if rc != SKY_OK:
        raise SkylineError(rc, ctx.error())
    res = BatchIds(out, list(offs))
    if return_stats:
        return res, {"n_total": st.n_total, "size_sky": st.size_sky, "n_groups": st.n_groups,
                     "ms_total": st.ms_total}
    return res


def tune_default(d: int) -> dict:
    """The built-in work splits of the dominance kernels for d coordinates."""
    t = SkyTuneParams()
    lib().sky_tune_default(int(d), C.byref(t))
    return t.as_dict()


def tune_get(d: int, n: int, ctx: Context | None = None) -> tuple[dict, bool]:
    """The splits a call with d coordinates and n points uses, and whether they come from the table."""
    ctx = ctx or context()
    t = SkyTuneParams()
    rc = lib().sky_tune_get(ctx.h, int(d), int(n), C.byref(t))
    if rc < 0:
        raise SkylineError(rc, "sky_tune_get")
    return t.as_dict(), rc == 1


def tune_set(d: int, n: int, params: dict, ctx: Context | None = None):
    """Set the table entry for (d, n); ``params`` holds the five fields of ``sky_tune_params``."""
    ctx = ctx or context()
    t = SkyTuneParams(**{k: int(params[k]) for k, _ in SkyTuneParams._fields_})
    rc = lib().sky_tune_set(ctx.h, int(d), int(n), C.byref(t))
    if rc != SKY_OK:
        raise SkylineError(rc, ctx.error())


def tune_clear(ctx: Context | None = None):
    lib().sky_tune_clear((ctx or context()).h)


def tune_save(path: str, ctx: Context | None = None):
    ctx = ctx or context()
    rc = lib().sky_tune_save(ctx.h, os.fsencode(path))
    if rc != SKY_OK:
        raise SkylineError(rc, f"sky_tune_save({path})")


def tune_load(path: str, ctx: Context | None = None):
    ctx = ctx or context()
    rc = lib().sky_tune_load(ctx.h, os.fsencode(path))
    if rc != SKY_OK:
        raise SkylineError(rc, ctx.error())


def autotune(points: torch.Tensor, trials: int = 5, ctx: Context | None = None, **opts) -> dict:
    """Tune the work splits for this input (``sky_autotune``) and store them in the context's
    table; ``opts`` are the keyword options of ``skyline``. Returns the splits and the median
    device times before and after."""
    _check_points(points)
    d, n = points.shape
    ctx = ctx or context(points.device.index)
    o = make_opts(**opts)
    t, best, base = SkyTuneParams(), C.c_float(0), C.c_float(0)
    rc = lib().sky_autotune(ctx.h, C.c_void_p(points.data_ptr()), n, d, C.byref(o), int(trials), C.byref(t),
                            C.byref(best), C.byref(base), _stream())
    if rc != SKY_OK:
        raise SkylineError(rc, ctx.error())
    return {"params": t.as_dict(), "best_ms": best.value, "base_ms": base.value}


def autotune_batch(packed: torch.Tensor, ns: list[int], ds: list[int], trials: int = 3,
                   ctx: Context | None = None, partitioning: str = "sliced", p: int = 16, reps: str = "sorted",
                   n_reps: int = 64, presort: str = "zorder") -> dict:
    """``sky_autotune_batch`` on a packed batch (``pack_instances`` layout)."""
    if len(ns) != len(ds) or not ns:
        raise ValueError("ns and ds must have one entry per instance")
    ctx = ctx or context(packed.device.index)
    o = make_opts(partitioning, p, None, 0, reps, n_reps, False, 0, "noseq", presort, None)
    n_inst = len(ns)
    ns_a = (C.c_int64 * n_inst)(*ns)
    ds_a = (C.c_int32 * n_inst)(*ds)
    t, best, base = SkyTuneParams(), C.c_float(0), C.c_float(0)
    rc = lib().sky_autotune_batch(ctx.h, C.c_void_p(packed.data_ptr()), ns_a, ds_a, n_inst, C.byref(o),
                                  int(trials), C.byref(t), C.byref(best), C.byref(base), _stream())
    if rc != SKY_OK:
        raise SkylineError(rc, ctx.error())
    return {"params": t.as_dict(), "best_ms": best.value, "base_ms": base.value}


def domby(points: torch.Tensor, by: torch.Tensor, ctx: Context | None = None) -> torch.Tensor:
    """Reverse dominance counts: out[i] = #{j : point by[j] dominates point i} (int32, device)."""
    _check_points(points)
    d, n = points.shape
    if by.dtype != torch.int32 or not by.is_cuda or not by.is_contiguous():
        raise ValueError("by must be a contiguous int32 device tensor of point ids")
    ctx = ctx or context(points.device.index)
    out = torch.empty(n, dtype=torch.int32, device=points.device)
    rc = lib().sky_domby(ctx.h, C.c_void_p(points.data_ptr()), n, d, C.c_void_p(by.data_ptr()), by.numel(),
                         C.c_void_p(out.data_ptr()), _stream())
    if rc != SKY_OK:
        raise SkylineError(rc, "sky_domby")
    return out


def mlp_targets(points: torch.Tensor, sample: torch.Tensor, reps: torch.Tensor | None = None,
                ctx: Context | None = None) -> tuple[torch.Tensor, int]:
    """Training targets of the scorer (float32 device tensor, one per point) from dominance
    counts against the sample points no point of ``reps`` dominates, and that residual
    sample's size: y = -log1p(dc * N / M) / log1p(N) (see ``sky_mlp_targets``)."""
    _check_points(points)
    d, n = points.shape
    for name, t in (("sample", sample), ("reps", reps)):
        if t is not None and (t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous int32 device tensor of point ids")
    ctx = ctx or context(points.device.index)
    y = torch.empty(n, dtype=torch.float32, device=points.device)
    kept = C.c_int64(0)
    nr = 0 if reps is None else reps.numel()
    rc = lib().sky_mlp_targets(ctx.h, C.c_void_p(points.data_ptr()), n, d, C.c_void_p(sample.data_ptr()),
                               sample.numel(), C.c_void_p(reps.data_ptr()) if nr else None, nr,
                               C.c_void_p(y.data_ptr()), C.byref(kept), _stream())
    if rc != SKY_OK:
        raise SkylineError(rc, "sky_mlp_targets")
    return y, int(kept.value)


def domcount(points: torch.Tensor, sample: torch.Tensor, ctx: Context | None = None) -> torch.Tensor:
    """Dominance counts (Def. 2): out[i] = #{j : point i dominates point sample[j]} (int32, device)."""
    _check_points(points)
    d, n = points.shape
    if sample.dtype != torch.int32 or not sample.is_cuda or not sample.is_contiguous():
        raise ValueError("sample must be a contiguous int32 device tensor of point ids")
    ctx = ctx or context(points.device.index)
    out = torch.empty(n, dtype=torch.int32, device=points.device)
    rc = lib().sky_domcount(ctx.h, C.c_void_p(points.data_ptr()), n, d, C.c_void_p(sample.data_ptr()),
                            sample.numel(), C.c_void_p(out.data_ptr()), _stream())
    if rc != SKY_OK:
        raise SkylineError(rc, "sky_domcount")
    return out


class Scorer:
    """The monotone MLP scorer d -> 64 -> 64 -> 1 (weights >= 0), trained on the GPU."""

    def __init__(self, d: int, init: torch.Tensor | None = None, seed: int = 0, ctx: Context | None = None,
                 _handle=None):
        self.ctx = ctx or context()
        self.d = int(d)
        self.nparams = int(lib().sky_mlp_nparams(self.d, MLP_HIDDEN))
        if _handle is not None:
            self.h = _handle
            return
        buf = None
        if init is not None:
            buf = torch.as_tensor(init, dtype=torch.float32).contiguous().cpu()
            if buf.numel() != self.nparams:
                raise ValueError(f"init must hold {self.nparams} parameters")
        h = C.c_void_p()
        rc = lib().sky_mlp_create(self.ctx.h, self.d, MLP_HIDDEN,
                                  C.c_void_p(buf.data_ptr()) if buf is not None else None, int(seed),
                                  C.byref(h))
        if rc != SKY_OK:
            raise SkylineError(rc, "sky_mlp_create")
        self.h = h

    @classmethod
    def load(cls, path: str, ctx: Context | None = None) -> "Scorer":
        ctx = ctx or context()
        h = C.c_void_p()
        rc = lib().sky_mlp_load(ctx.h, path.encode(), C.byref(h))
        if rc != SKY_OK:
            raise SkylineError(rc, f"sky_mlp_load({path})")
        with open(path, "rb") as f:   # the file header holds d after the 8-byte magic
            hdr = f.read(16)
        return cls(int.from_bytes(hdr[8:12], "little", signed=True), ctx=ctx, _handle=h)

    def save(self, path: str):
        rc = lib().sky_mlp_save(self.h, path.encode())
        if rc != SKY_OK:
            raise SkylineError(rc, f"sky_mlp_save({path})")

    def params(self) -> torch.Tensor:
        out = torch.empty(self.nparams, dtype=torch.float32)
        rc = lib().sky_mlp_get_params(self.h, C.c_void_p(out.data_ptr()), self.nparams)
        if rc != SKY_OK:
            raise SkylineError(rc, "sky_mlp_get_params")
        return out

    def score(self, points: torch.Tensor) -> torch.Tensor:
        _check_points(points)
        d, n = points.shape
        out = torch.empty(n, dtype=torch.float32, device=points.device)
        rc = lib().sky_mlp_score(self.ctx.h, self.h, C.c_void_p(points.data_ptr()), n, d,
                                 C.c_void_p(out.data_ptr()), _stream())
        if rc != SKY_OK:
            raise SkylineError(rc, "sky_mlp_score")
        return out

    def loss_grad(self, points: torch.Tensor, y: torch.Tensor):
        _check_points(points)
        d, n = points.shape
        y = y.to(device=points.device, dtype=torch.float32).contiguous()
        grad = torch.empty(self.nparams, dtype=torch.float32, device=points.device)
        loss = torch.empty(1, dtype=torch.float32, device=points.device)
        rc = lib().sky_mlp_loss_grad(self.ctx.h, self.h, C.c_void_p(points.data_ptr()), n, d,
                                     C.c_void_p(y.data_ptr()), C.c_void_p(grad.data_ptr()),
                                     C.c_void_p(loss.data_ptr()), _stream())
        if rc != SKY_OK:
            raise SkylineError(rc, "sky_mlp_loss_grad")
        return loss, grad

    def adam_step(self, grad: torch.Tensor, lr: float, step: int, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8):
        g = grad.to(dtype=torch.float32).contiguous()
        rc = lib().sky_mlp_adam_step(self.ctx.h, self.h, C.c_void_p(g.data_ptr()), lr, beta1, beta2, eps,
                                     int(step), _stream())
        if rc != SKY_OK:
            raise SkylineError(rc, "sky_mlp_adam_step")

    def train(self, points: torch.Tensor, y: torch.Tensor, epochs: int = 1, batch: int = 4096,
              lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> float:
        _check_points(points)
        d, n = points.shape
        y = y.to(device=points.device, dtype=torch.float32).contiguous()
        to = SkyTrainOpts(epochs, batch, lr, beta1, beta2, eps)
        loss = C.c_float(0.0)
        rc = lib().sky_mlp_train(self.ctx.h, self.h, C.c_void_p(points.data_ptr()), n, d,
                                 C.c_void_p(y.data_ptr()), C.byref(to), C.byref(loss), _stream())
        if rc != SKY_OK:
            raise SkylineError(rc, "sky_mlp_train")
        return float(loss.value)

    def close(self):
        if getattr(self, "h", None):
            lib().sky_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
