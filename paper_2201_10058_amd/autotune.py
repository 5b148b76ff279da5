"""Self-tuning of kick launch shapes (cf. the self-tuning kernel parameters of
GENGA II, Sect. 8): candidate shapes are timed on the caller's own inputs and
the fastest is kept, cached in a JSON file keyed by device architecture,
precision and problem signature.

Timing runs the kick with a zero step factor and no encounter list, so the
caller's state is not modified.
"""
from __future__ import annotations

import json
import os
import statistics

import numpy as np
import torch

from . import native as N

CACHE_ENV = "GENGA_TUNE_CACHE"


def _cache_path() -> str:
    p = os.environ.get(CACHE_ENV)
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "genga_mi355x", "autotune.json")


def _load_cache() -> dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(c: dict) -> None:
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    except OSError:
        pass


def _arch() -> str:
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def _time(fn, reps: int = 3) -> float:
    fn()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return statistics.median(ts)


def batch_signature(batch: N.Batch) -> str:
    sizes = np.diff(batch.offsets)
    hist = np.histogram(np.log2(sizes), bins=8, range=(0, 16))[0]
    return f"S{batch.S}-N{batch.n}-h{'.'.join(map(str, hist))}"


BATCH_CANDIDATES = [dict(block=b, ipt=i, tile_cols=c)
                    for b in (64, 256) for i in (1, 2) for c in (256, 512, 1024, 2048)]


def _batch_candidates() -> list:
    """Tile shapes, each with the library's occupancy-sized persistent grid
    (grid = 0) and with a grid of 32 waves per CU."""
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    out = []
    for c in BATCH_CANDIDATES:
        out.append({**c, "grid": 0})
        out.append({**c, "grid": cus * (32 * 64 // c["block"])})
    return out


def tune_batched(state: N.State, batch: N.Batch, cfg: N.Config, use_cache: bool = True,
                 candidates=None, reps: int = 3) -> dict:
    """Pick (block, ipt, tile_cols, grid) for the batched kick; returns the choice."""
    key = f"batch2:{_arch()}:p{cfg.precision}:{batch_signature(batch)}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return cache[key]["choice"]
    results = []
    for cand in candidates or _batch_candidates():
        c = N.Config(**{**cfg.__dict__, **cand, "flags": N.FLAG_NOSYNC})
        ws = N.BatchWorkspace(batch, c)
        ms = _time(lambda: N.kick_batched(state, ws, c, 0.0), reps)
        results.append((ms, cand))
        del ws
    results.sort(key=lambda r: r[0])
    choice = dict(results[0][1])
    if use_cache:
        cache[key] = {"choice": choice, "ms": results[0][0],
                      "tried": [{"ms": m, **c} for m, c in results]}
        _store_cache(cache)
    return choice


SINGLE_CANDIDATES = [dict(ipt=i, slices=s) for i in (1, 2) for s in (8, 16, 32, 64)]


def tune_single(state: N.State, cfg: N.Config, use_cache: bool = True, candidates=None,
                reps: int = 3) -> dict:
    """Pick (ipt, slices) for the single-system kick of this size."""
    bucket = 1 << max(0, int(np.ceil(np.log2(max(state.n, 1)))))
    key = f"single:{_arch()}:p{cfg.precision}:N{bucket}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return cache[key]["choice"]
    results = []
    for cand in candidates or SINGLE_CANDIDATES:
        c = N.Config(**{**cfg.__dict__, **cand})
        ws = N.Workspace(state.n, c)
        ms = _time(lambda: N.kick(state, c, ws, 0.0), reps)
        results.append((ms, cand))
        del ws
    results.sort(key=lambda r: r[0])
    choice = dict(results[0][1])
    if use_cache:
        cache[key] = {"choice": choice, "ms": results[0][0],
                      "tried": [{"ms": m, **c} for m, c in results]}
        _store_cache(cache)
    return choice
