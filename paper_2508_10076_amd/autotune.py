"""Tile-configuration autotuner for the grouped sector GEMM.

For a plan (or a batch of plans) every tile configuration the library
offers, (tile_m, tile_n, tile_k), is applied in turn (the library
re-schedules the tiles, split-K included) and the GEMM stage is timed with
HIP events on the caller's stream; the fastest is kept.  Winners are cached
in a JSON file keyed by a shape class of the sector-GEMM list, so later runs
with the same class skip the search.
"""
from __future__ import annotations

import json
import math
import os

from . import tk

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_tiles.json")


def shape_class(mnk, dtype="f64", precision="native") -> str:
    """Coarse signature of a list of sector GEMM shapes: count, log2 of the
    largest M, N, K and of the total flops (MFMA-sized GEMMs only)."""
    big = [(m, n, k) for m, n, k in mnk if k > 8]
    if not big:
        return f"{dtype}/{precision}/none"
    lg = lambda x: int(round(math.log2(max(1, x))))
    mx = [max(x[i] for x in big) for i in range(3)]
    fl = sum(2 * m * n * k for m, n, k in big)
    return f"{dtype}/{precision}/g{lg(len(big))}/m{lg(mx[0])}n{lg(mx[1])}k{lg(mx[2])}/f{lg(fl)}"


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save(path, data):
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_ms(run, stream, reps):
    import torch
    with torch.cuda.stream(stream):
        run()
    stream.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        run()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def lookup(mnk, tag=("f64", "native"), cache_path=DEFAULT_CACHE):
    """The cached winner for this shape class, or None (never times, never
    writes the cache)."""
    ent = _load(cache_path).get(shape_class(mnk, *tag))
    return tuple(ent["tile"]) if ent else None


def tune(target, run, mnk, stream, cache_path=DEFAULT_CACHE, reps=5, force=False, tag=("f64", "native")):
    """target: a tk.Plan or tk.Batch; run(): enqueues its GEMM work on
    `stream`.  Returns (best_config, {config: ms})."""
    key = shape_class(mnk, *tag)
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        cfg = tuple(cache[key]["tile"])
        target.set_tile(*cfg)
        times = {tuple(int(x) for x in c.split("x")): t for c, t in cache[key].get("times", {}).items()}
        return cfg, times
    times = {}
    for cfg in tk.tile_shapes():
        try:
            target.set_tile(*cfg)
        except tk.TkError:
            continue
        times[cfg] = _time_ms(run, stream, reps)
    best = min(times, key=times.get)
    target.set_tile(*best)
    if cache_path:
        cache = _load(cache_path)
        cache[key] = {"tile": list(best), "times": {"x".join(map(str, c)): round(t, 4) for c, t in times.items()}}
        _save(cache_path, cache)
    return best, times
