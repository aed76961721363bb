"""Autotuner for the launch settings of the batched path.

The settings (see ``hop_tuning`` in the C header) change speed, never
results: the kNN walk's frontier cap, whether the persistent launch keeps
one work chunk per XCD, and whether subvolumes are taken largest first.
The tuner times every candidate on the caller's own batch and keeps the
fastest, cached in a JSON file per size class so that batches of a similar
shape reuse it.
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time

__all__ = ["SPACE", "size_class", "default_cache_path", "tune_batch", "load_cache"]

# candidate values of each setting
SPACE = {
    "front_cap": [256, 512, 1024],
    "xcd_queues": [0, 1],
    "largest_first": [0, 1],
}


def size_class(offsets) -> str:
    """Batches whose total size and subvolume count round to the same powers
    of two share a cache entry."""
    off = [int(v) for v in offsets]
    n_sub = len(off) - 1
    total = off[-1] - off[0]
    if n_sub < 1 or total <= 0:
        raise ValueError("offsets must describe at least one non-empty subvolume")
    return f"n2^{round(math.log2(total))}_sub2^{round(math.log2(n_sub))}"


def default_cache_path() -> str:
    return os.environ.get("HOP_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "hop_tuning.json"))


def load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _save_cache(path: str, data: dict) -> None:
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def candidates(space: dict | None = None):
    space = space or SPACE
    keys = sorted(space)
    for vals in itertools.product(*(space[k] for k in keys)):
        yield dict(zip(keys, vals))


def tune_batch(ctx, pos, offsets, params, padded=None, mean_density=None, reps: int = 2,
               cache_path: str | None = None, space: dict | None = None, sync=None,
               force: bool = False) -> dict:
    """Pick and apply the fastest launch settings for this batch shape.

    ctx: a HopContext (anything with run_batch / set_tuning); sync: called
    before reading the clock (torch.cuda.synchronize by default).  Returns
    {"tuning": best settings, "ms": its time, "trials": [...], "cached": bool}.
    """
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    path = cache_path or default_cache_path()
    key = size_class(offsets)
    cache = load_cache(path)
    if not force and key in cache and isinstance(cache[key], dict) and "tuning" in cache[key]:
        ctx.set_tuning(**cache[key]["tuning"])
        return {**cache[key], "cached": True}
    trials = []
    for cand in candidates(space):
        ctx.set_tuning(**cand)
        ctx.run_batch(pos, offsets, params, padded=padded, mean_density=mean_density)  # warm
        best = math.inf
        for _ in range(max(1, reps)):
            sync()
            t0 = time.perf_counter()
            ctx.run_batch(pos, offsets, params, padded=padded, mean_density=mean_density)
            sync()
            best = min(best, (time.perf_counter() - t0) * 1e3)
        trials.append({"tuning": cand, "ms": best})
    win = min(trials, key=lambda t: t["ms"])
    ctx.set_tuning(**win["tuning"])
    entry = {"tuning": win["tuning"], "ms": win["ms"], "trials": trials}
    cache[key] = entry
    _save_cache(path, cache)
    return {**entry, "cached": False}
