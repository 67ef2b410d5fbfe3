"""Autotuner for the launch knobs of the evaluation kernels.

The knobs change how work is cut, never what is computed (the tests check that every candidate
gives the same outputs):

* per register class of a RANGE evaluation (``class_seg_tiles``, ``class_lanes`` of
  ``thoi_eval_opts``): tiles of 256 lanes walked by one workgroup (amortises the staging of the
  correlation matrix and the binomial table against fewer, longer workgroups), and n-plets per
  lane (1, or 2 where the class has register room: the second is reached by the lexicographic
  successor, so the unranking is paid once per pair, at the price of registers);
* for the multi-dataset path, ``seg_tiles`` (units per workgroup) and ``grid_blocks`` (workgroups
  of the persistent class launches).

The tuner times every candidate on the caller's problem with HIP events around a HIP graph of
repeated calls, keeps the fastest, and caches the choice in a JSON file keyed by (GPU
architecture, path, precision, register class, N bucket, dataset-count bucket).  ``Evaluator``
and ``MultiEvaluator`` look the cache up whenever they are created without explicit knobs.

The split of orders into register classes is fixed at compile time (one kernel per class); the
alternative splits that were measured are recorded in the design notes.
"""
from __future__ import annotations

import json
import os

import torch

from . import api
from . import binding as B

_CACHE_ENV = "THOI_TUNE_CACHE"

# Register classes of the lane engine per precision (the library's class tables) and whether the
# class has room for two n-plets per lane in RANGE mode.
CLASSES = {
    "fp32": [(0, 8), (9, 12), (13, 16), (17, 20), (21, 24)],
    "fp64": [(0, 6), (7, 10), (11, 14), (15, 18)],
}
_PAIR_ROOM = {"fp32": 16, "fp64": 10}
_NAMES = {B.THOI_FP64: "fp64", B.THOI_FP32: "fp32", B.THOI_FP32_REFINE: "fp32_refine"}


def _table(precision: str) -> str:
    return "fp64" if precision == "fp64" else "fp32"


def n_bucket(N: int) -> str:
    for hi in (12, 16, 24, 32, 48, 62):
        if N <= hi:
            return f"N<={hi}"
    return "N>62"


def d_bucket(D: int) -> str:
    for hi in (1, 8, 64):
        if D <= hi:
            return f"D<={hi}"
    return "D>64"


def range_key(arch: str, precision: str, cls: int, N: int, D: int) -> str:
    lo, hi = CLASSES[_table(precision)][cls]
    return f"{arch}|range|{precision}|k{lo}-{hi}|{n_bucket(N)}|{d_bucket(D)}"


def multi_key(arch: str, precision: str, N_d, kmin: int, kmax: int) -> str:
    return f"{arch}|multi|{precision}|{n_bucket(int(max(N_d)))}|{d_bucket(len(N_d))}|k{kmin}-{kmax}"


def _cache_path() -> str:
    return os.environ.get(_CACHE_ENV, os.path.join(os.path.expanduser("~"), ".cache", "thoi_tune.json"))


def _load_cache() -> dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(c: dict) -> None:
    p = _cache_path()
    try:
        os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
        with open(p, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
    except OSError:
        pass


def _arch(device) -> str:
    if isinstance(device, str) and not device.startswith("cuda"):
        return device
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def lookup_range(device, precision, N: int, D: int):
    """(class_seg_tiles[8], class_lanes[8]) cached for a RANGE evaluation of this shape, or None
    when no class of it has been tuned.  precision: a name or a THOI_* value; device: a torch
    device or an architecture name."""
    prec = _NAMES.get(precision, precision)
    cache = _load_cache()
    if not cache:
        return None
    arch = _arch(device)
    seg, lanes, hit = [0] * 8, [0] * 8, False
    for c in range(len(CLASSES[_table(prec)])):
        e = cache.get(range_key(arch, prec, c, N, D))
        if e:
            seg[c], lanes[c], hit = int(e["seg_tiles"]), int(e["lanes"]), True
    return (seg, lanes) if hit else None


def lookup_multi(device, precision, N_d, kmin: int, kmax: int):
    """(seg_tiles, grid_blocks) cached for the multi-dataset path on datasets of this shape, or None."""
    prec = _NAMES.get(precision, precision)
    e = _load_cache().get(multi_key(_arch(device), prec, N_d, kmin, kmax))
    return (int(e["seg_tiles"]), int(e["grid_blocks"])) if e else None


def time_call(fn, device, reps: int = 10, trials: int = 3) -> float:
    """Milliseconds per call of fn(stream_handle), from HIP events around a graph of `reps` calls."""
    stream = torch.cuda.Stream(device)
    with torch.cuda.stream(stream):
        fn(stream.cuda_stream)
    torch.cuda.synchronize(device)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        h = torch.cuda.current_stream(device).cuda_stream
        for _ in range(reps):
            fn(h)
    torch.cuda.synchronize(device)
    best = float("inf")
    for _ in range(trials):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            e0.record(stream)
            g.replay()
            e1.record(stream)
        torch.cuda.synchronize(device)
        best = min(best, e0.elapsed_time(e1) / reps)
    return best


def tune_range(Sigma: torch.Tensor, kmin: int, kmax: int, precision: str = "fp32_refine",
               seg_candidates=(1, 2, 4, 8), use_cache: bool = True) -> dict:
    """Best (tiles per workgroup, n-plets per lane) of every register class that orders kmin..kmax
    of a RANGE evaluation on Sigma [D, N, N] touch; each class is timed alone on its own orders."""
    S = Sigma if Sigma.dim() == 3 else Sigma[None]
    D, N, _ = S.shape
    arch = _arch(S.device)
    table = _table(precision)
    lane_max = CLASSES[table][-1][1]
    odt = torch.float64 if precision == "fp64" else torch.float32
    cache = _load_cache() if use_cache else {}
    seg, lanes, detail = [0] * 8, [0] * 8, {}
    for c, (lo, hi) in enumerate(CLASSES[table]):
        k0, k1 = max(lo, kmin), min(hi, kmax, N, lane_max)
        if k0 > k1:
            continue
        key = range_key(arch, precision, c, N, D)
        if key in cache:
            seg[c], lanes[c] = int(cache[key]["seg_tiles"]), int(cache[key]["lanes"])
            detail[key] = cache[key]
            continue
        sel = api.range_selection(N, k0, k1)
        lane_choices = (0, 1) if hi <= _PAIR_ROOM[table] else (0,)
        timings = {}
        for st in seg_candidates:
            for ln in lane_choices:
                cs, cl = [0] * 8, [0] * 8
                cs[c], cl[c] = st, ln
                opts = api.make_opts(precision, odt, class_seg_tiles=cs, class_lanes=cl)
                ev = api.Evaluator(D, N, sel, opts, S.device, odt, tuned=False)
                timings[(st, ln)] = time_call(lambda h: ev(S, stream=h), S.device)
        best = min(timings, key=timings.get)
        seg[c], lanes[c] = best
        detail[key] = {"seg_tiles": int(best[0]), "lanes": int(best[1]), "ms": timings[best],
                       "timings_ms": {f"{a},{b}": v for (a, b), v in timings.items()}}
        if use_cache:
            cache[key] = detail[key]
    if use_cache:
        _store_cache(cache)
    return {"class_seg_tiles": seg, "class_lanes": lanes, "classes": detail}


def tune_multi(Sigma_packed: torch.Tensor, N_d, kmin: int, kmax: int, precision: str = "fp32_refine",
               seg_candidates=(1, 2, 4, 8), grid_candidates=(0, 512, 1024, 2048), use_cache: bool = True) -> dict:
    """Best (seg_tiles, grid_blocks) for the multi-dataset path on the given datasets."""
    import numpy as np
    Nd = np.asarray(N_d, dtype=np.int32)
    key = multi_key(_arch(Sigma_packed.device), precision, Nd, kmin, kmax)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return cache[key]
    odt = torch.float64 if precision == "fp64" else torch.float32
    timings = {}
    for st in seg_candidates:
        for gb in grid_candidates:
            ev = api.MultiEvaluator(Nd, kmin, kmax, Sigma_packed.device, precision, odt, seg_tiles=st,
                                    grid_blocks=gb)
            timings[(st, gb)] = time_call(lambda h: ev(Sigma_packed, stream=h), Sigma_packed.device)
    best = min(timings, key=timings.get)
    res = {"seg_tiles": int(best[0]), "grid_blocks": int(best[1]), "ms": timings[best],
           "timings_ms": {f"{a},{b}": v for (a, b), v in timings.items()}}
    if use_cache:
        cache[key] = res
        _store_cache(cache)
    return res
