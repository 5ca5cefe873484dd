"""Tile-shape x LDS-batch autotuner for the batched chunk.

Every candidate (tile shape, staging batch) is applied to the context and the
whole chunk is run and timed with HIP events on the current stream; the
fastest median wins.  Results are cached per workload key in a JSON file
(default ~/.cache/kgs_autotune.json) so that a later run of the same shape
can skip the search.
"""
from __future__ import annotations

import json
import os
from typing import Callable, Iterable, Optional

import numpy as np
import torch

CACHE = os.path.join(os.path.expanduser("~"), ".cache", "kgs_autotune.json")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def autotune(run: Callable[[], None], set_tiling: Callable, tiles: Iterable, batches: Iterable, reps: int = 3,
             warmup: int = 1, key: Optional[str] = None, cache_path: Optional[str] = CACHE):
    """Return ((tile_w, tile_h), batch) of the fastest candidate and the table
    {"WxH/B": median ms}."""
    if key and cache_path:
        hit = _load(cache_path).get(key)
        if hit:
            return (tuple(hit["tile"]), int(hit["batch"])), hit.get("table")
    stream = torch.cuda.current_stream()
    table = {}
    best, best_ms = None, float("inf")
    for tile in tiles:
        for b in batches:
            if tile[0] * tile[1] == 512 and b > 64:
                continue  # not a valid tiling (at most 64 records per stage with 512-pixel tiles)
            set_tiling(tuple(tile), int(b))
            for _ in range(warmup):
                run()
            times = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                run()
                e1.record(stream)
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            ms = float(np.median(times))
            table[f"{tile[0]}x{tile[1]}/{b}"] = round(ms, 4)
            if ms < best_ms:
                best, best_ms = (tuple(tile), int(b)), ms
    if key and cache_path:
        data = _load(cache_path)
        data[key] = {"tile": list(best[0]), "batch": best[1], "table": table}
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            with open(cache_path, "w") as f:
                json.dump(data, f, indent=1)
        except OSError:
            pass
    return best, table
