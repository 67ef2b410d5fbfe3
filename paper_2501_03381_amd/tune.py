"""Autotuner for the launch knobs of the evaluation kernels.

Two knobs of ``thoi_eval_opts`` change how work is cut, not what is computed:

* ``seg_tiles``  - tiles of 256 n-plets walked by one workgroup (amortises the staging of the
  correlation matrix and the binomial table; fewer, longer workgroups);
* ``grid_blocks`` - workgroups of a persistent launch (multi-dataset path).

The tuner times every candidate on the caller's actual problem with HIP events around a HIP
graph of repeated calls, keeps the fastest, and caches the choice in a JSON file keyed by
(GPU architecture, path, precision, N or N-range, orders).  Results are identical for every
candidate (the tests check this), so tuning never changes numbers.
"""
from __future__ import annotations

import ctypes
import json
import os

import torch

from . import api
from . import binding as B

_CACHE_ENV = "THOI_TUNE_CACHE"


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
        os.makedirs(os.path.dirname(p), exist_ok=True)
        with open(p, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
    except OSError:
        pass


def _arch(device) -> str:
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


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
               candidates=(1, 2, 4, 8), use_cache: bool = True) -> dict:
    """Best seg_tiles for an exhaustive RANGE evaluation of orders kmin..kmax on Sigma [D, N, N]."""
    S = Sigma if Sigma.dim() == 3 else Sigma[None]
    D, N, _ = S.shape
    key = f"{_arch(S.device)}|range|{precision}|D{D}|N{N}|k{kmin}-{kmax}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return cache[key]
    odt = torch.float64 if precision == "fp64" else torch.float32
    sel = api.range_selection(N, kmin, kmax)
    timings = {}
    for st in candidates:
        opts = api.make_opts(precision, odt, seg_tiles=st)
        ev = api.Evaluator(D, N, sel, opts, S.device, odt)
        timings[st] = time_call(lambda h: ev(S, stream=h), S.device)
    best = min(timings, key=timings.get)
    res = {"seg_tiles": int(best), "ms": timings[best], "timings_ms": {str(k): v for k, v in timings.items()}}
    if use_cache:
        cache[key] = res
        _store_cache(cache)
    return res


def tune_multi(Sigma_packed: torch.Tensor, N_d, kmin: int, kmax: int, precision: str = "fp32_refine",
               seg_candidates=(1, 2, 4, 8), grid_candidates=(0, 512, 1024, 2048), use_cache: bool = True) -> dict:
    """Best (seg_tiles, grid_blocks) for the multi-dataset path on the given datasets."""
    import numpy as np
    Nd = np.asarray(N_d, dtype=np.int32)
    key = (f"{_arch(Sigma_packed.device)}|multi|{precision}|D{len(Nd)}|N{int(Nd.min())}-{int(Nd.max())}"
           f"|sum{int(Nd.sum())}|k{kmin}-{kmax}")
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
