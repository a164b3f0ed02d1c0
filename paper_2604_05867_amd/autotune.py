"""Autotuner for the launch parameters of libba.

For a workload (input lengths, iteration precision, engine) it times a few BA
iterations per candidate setting of the tuning knobs (``ba_set_tuning``) with HIP
events on the bound stream (``ba_time_kernels``), and keeps the fastest.  The knobs
are searched one after another (coordinate descent from the library defaults:
each knob tries all its values with the others at their best so far), and the
choice is cached in a JSON file keyed by device and workload.  The knobs only
change the work decomposition, never the results beyond rounding order.

Knobs:
  engine factored:
    TUNE_FACTORED_FUSE     positions per launch (launch plan level 8 .. 0)
    TUNE_STAGE8_COLUMNS    columns per block of the eight-position backward
                           launches, log2 (0 = widest, 1 .. 4), i.e. the tile of
                           (subtree roots x columns) a block stages in LDS
    TUNE_PERSISTENT        small groups as one persistent launch (auto, off, always)
    TUNE_PERSIST_THREADS   threads per block of that launch (1024, 512, 256)
  engine stream:
    TUNE_SCATTER_LDS_KB    LDS-privatised output range of the scatter (KB)
"""
from __future__ import annotations

import json
import os

import torch

from . import (ENGINE_FACTORED, ENGINE_STREAM, TUNE_FACTORED_FUSE, TUNE_PERSIST_THREADS, TUNE_PERSISTENT,
               TUNE_SCATTER_LDS_KB, TUNE_STAGE8_COLUMNS, Context)

# knob -> candidate values, the library default first
KNOBS = {
    ENGINE_FACTORED: [(TUNE_FACTORED_FUSE, [8, 7, 6, 5, 4, 3, 2, 1, 0]),
                      (TUNE_STAGE8_COLUMNS, [0, 1, 2, 3, 4]),
                      (TUNE_PERSISTENT, [1, 0, 2]),
                      (TUNE_PERSIST_THREADS, [1024, 512, 256])],
    ENGINE_STREAM: [(TUNE_SCATTER_LDS_KB, [64, 48, 32, 16])],
}


def _key(ns, prec, engine):
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    return "%s|n=%s|prec=%d|engine=%d" % (dev, ",".join(str(v) for v in sorted(set(ns))), prec, engine)


def _apply(ctx: Context, choice: dict):
    for knob, value in choice.items():
        ctx.set_tuning(int(knob), int(value))


def _time(ctx: Context, start: torch.Tensor, iters: int) -> float:
    ctx.set_logp(start)
    ctx.step(1)  # warm-up (first launch of a new shape)
    t = ctx.time_kernels(iters)
    return sum(ms for ms, _ in t.values()) / iters


def tune(ctx: Context, iters: int = 3, cache_path: str | None = None, force: bool = False,
         margin: float = 0.02) -> dict:
    """Choose and apply the fastest knob settings for ``ctx``'s workload.

    Returns {"key", "choice": {knob: value}, "ms_per_iter": {"knob=value": ms}}.
    The timing runs ``iters`` iterations per candidate on the context itself and
    then restores the starting iterate.  A candidate replaces the current choice
    only if it is faster by more than ``margin`` (relative), so that timing noise
    does not move a knob away from its default."""
    if ctx.engine not in KNOBS:
        return {"key": None, "choice": {}, "ms_per_iter": {}}
    key = _key(ctx.n, ctx.prec, ctx.engine)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key in cache and not force:
        _apply(ctx, cache[key]["choice"])
        return cache[key]
    start = ctx.get_logp()
    choice = {str(knob): values[0] for knob, values in KNOBS[ctx.engine]}
    _apply(ctx, choice)
    results = {}
    best_ms = None
    for knob, values in KNOBS[ctx.engine]:
        for value in values:
            trial = dict(choice)
            trial[str(knob)] = value
            label = "%d=%d" % (knob, value)
            if label not in results:
                _apply(ctx, trial)
                results[label] = _time(ctx, start, iters)
            if best_ms is None:
                best_ms = results[label]
            elif results[label] < best_ms * (1.0 - margin):
                best_ms = results[label]
                choice = trial
        _apply(ctx, choice)
    _apply(ctx, choice)
    ctx.set_logp(start)
    entry = {"key": key, "choice": choice, "ms_per_iter": results}
    if cache_path:
        cache[key] = entry
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return entry
