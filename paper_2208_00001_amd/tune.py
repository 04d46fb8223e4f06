"""Autotuner for the batched launch.

Times candidate schedules of a batch (chunk length K, i.e. the halo depth and
the number of scan steps between neighbour exchanges; the 3D tile side, 16 or
24 for single-channel volumes; and the number of co-resident workgroups
planned per compute unit) with HIP-graph replays and keeps the fastest.  Results are cached in a JSON file keyed by the batch's shape
signature (GGDT_TUNE_CACHE, default ~/.cache/ggdt_tune.json).
"""
from __future__ import annotations

import json
import os
from typing import Optional, Sequence

import torch

CANDIDATES = (
    {"chunk": 8, "wg_per_cu": 1},
    {"chunk": 8, "wg_per_cu": 0},
    {"chunk": 4, "wg_per_cu": 1},
    {"chunk": 4, "wg_per_cu": 2},
    {"chunk": 4, "wg_per_cu": 0},
    {"chunk": 4, "tile_p": 24, "wg_per_cu": 1},
    {"chunk": 4, "tile_p": 24, "wg_per_cu": 0},
)


def cache_path() -> str:
    return os.environ.get("GGDT_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "ggdt_tune.json"))


def signature(instances: Sequence[dict]) -> str:
    """Shape class of a batch: per instance (ndim, C, dims rounded up to 32,
    iterations, lambda class), order-independent."""
    items = []
    for d in instances:
        m = d["softmask"]
        img = d["image"]
        C = img.shape[0] if img.dim() > m.dim() else 1
        lam = float(d["lam"])
        lam_cls = "0" if lam == 0.0 else ("1" if lam == 1.0 and C == 1 else "g")
        dims = tuple(-(-int(s) // 32) * 32 for s in m.shape)
        items.append((m.dim(), C, dims, int(d["iterations"]), lam_cls))
    items.sort()
    return json.dumps(items)


def _load_cache():
    p = cache_path()
    if os.path.exists(p):
        try:
            with open(p) as f:
                return json.load(f)
        except (OSError, ValueError):
            return {}
    return {}


def _save_cache(c):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def time_plan(plan, reps: int = 5, warmup: int = 2) -> float:
    """Median ms of graph replays of a BatchedPlan."""
    plan.capture()
    for _ in range(warmup):
        plan.replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        plan.replay()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    if plan.status() != 0:
        raise RuntimeError("watchdog fired while tuning")
    times.sort()
    return times[len(times) // 2]


def tune(instances: Sequence[dict], candidates=CANDIDATES, reps: int = 5, use_cache: bool = True,
         verbose: bool = False) -> dict:
    """Best tuning for this batch (from the cache when known).  Returns
    {"tuning": {...}, "ms": best, "trials": {...}}."""
    from .batched import BatchedPlan
    from .binding import GGDTError

    sig = signature(instances)
    cache = _load_cache() if use_cache else {}
    if sig in cache:
        return cache[sig]
    trials = {}
    best = None
    for cand in candidates:
        key = json.dumps(cand, sort_keys=True)
        try:
            plan = BatchedPlan(instances, cand)
        except GGDTError as e:  # candidate not valid for this batch (e.g. too many channels for the chunk)
            trials[key] = str(e)
            continue
        try:
            ms = time_plan(plan, reps)
        finally:
            plan.close()
        trials[key] = ms
        if verbose:
            print(f"tune {cand}: {ms:.3f} ms", flush=True)
        if best is None or ms < best[1]:
            best = (cand, ms)
    if best is None:
        raise RuntimeError(f"no candidate schedule is valid for this batch: {trials}")
    res = {"tuning": best[0], "ms": best[1], "trials": trials}
    if use_cache:
        cache[sig] = res
        _save_cache(cache)
    return res


def tuned_plan(instances: Sequence[dict], **kw):
    """A BatchedPlan with the autotuned schedule."""
    from .batched import BatchedPlan
    return BatchedPlan(instances, tune(instances, **kw)["tuning"])
