"""Autotuner for the launch parameters of libba.

For a workload (input lengths, iteration precision, engine) it times a few BA
iterations for every candidate setting of the tuning knobs (``ba_set_tuning``)
with HIP events on the bound stream (``ba_time_kernels``), keeps the fastest,
and caches the choice in a JSON file keyed by device and workload.  The knobs
only change the work decomposition, never the results beyond rounding order.

Knobs:
  engine factored: TUNE_FACTORED_FUSE in {0, 1, 2, 3, 4, 5} (positions per launch)
  engine stream:   TUNE_SCATTER_LDS_KB in {16, 32, 48, 64} (LDS-privatised
                   output range of the scatter)
"""
from __future__ import annotations

import json
import os

import torch

from . import (ENGINE_FACTORED, ENGINE_STREAM, TUNE_FACTORED_FUSE, TUNE_SCATTER_LDS_KB, Context)

CANDIDATES = {
    ENGINE_FACTORED: [(TUNE_FACTORED_FUSE, 0), (TUNE_FACTORED_FUSE, 1), (TUNE_FACTORED_FUSE, 2),
                      (TUNE_FACTORED_FUSE, 3), (TUNE_FACTORED_FUSE, 4), (TUNE_FACTORED_FUSE, 5)],
    ENGINE_STREAM: [(TUNE_SCATTER_LDS_KB, 16), (TUNE_SCATTER_LDS_KB, 32), (TUNE_SCATTER_LDS_KB, 48),
                    (TUNE_SCATTER_LDS_KB, 64)],
}


def _key(ns, prec, engine):
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    return "%s|n=%s|prec=%d|engine=%d" % (dev, ",".join(str(v) for v in sorted(set(ns))), prec, engine)


def tune(ctx: Context, iters: int = 3, cache_path: str | None = None, force: bool = False) -> dict:
    """Choose and apply the fastest knob setting for ``ctx``'s workload.

    Returns {"key", "choice": (knob, value), "ms_per_iter": {value: ms}}.  The
    timing runs ``iters`` iterations per candidate on the context itself and then
    restores the starting iterate."""
    if ctx.engine not in CANDIDATES:
        return {"key": None, "choice": None, "ms_per_iter": {}}
    key = _key(ctx.n, ctx.prec, ctx.engine)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key in cache and not force:
        knob, value = cache[key]["choice"]
        ctx.set_tuning(knob, value)
        return cache[key]
    start = ctx.get_logp()
    results = {}
    for knob, value in CANDIDATES[ctx.engine]:
        ctx.set_tuning(knob, value)
        ctx.set_logp(start)
        ctx.step(1)  # warm-up (first launch with new LDS size / shape)
        t = ctx.time_kernels(iters)
        results[value] = sum(ms for ms, _ in t.values()) / iters
    best = min(results, key=results.get)
    knob = CANDIDATES[ctx.engine][0][0]
    ctx.set_tuning(knob, best)
    ctx.set_logp(start)
    entry = {"key": key, "choice": [knob, best], "ms_per_iter": {str(k): v for k, v in results.items()}}
    if cache_path:
        cache[key] = entry
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return entry
