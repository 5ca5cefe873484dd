"""Tile-shape x LDS-batch autotuner for the batched chunk.

Every candidate (tile shape, staging batch) is applied to the context and the
whole chunk is run and timed with HIP events on the current stream.  The
few fastest candidates are then timed again, in turn (round robin, so that a
drift of the clock over the search touches each alike), with more repetitions;
the fastest median of that second pass wins.  Results are cached per workload key in a JSON file
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


def _time(run, stream):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    run()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def autotune(run: Callable[[], None], set_tiling: Callable, tiles: Iterable, batches: Iterable, reps: int = 3,
             warmup: int = 1, key: Optional[str] = None, cache_path: Optional[str] = CACHE, finalists: int = 3,
             final_rounds: int = 5):
    """Return ((tile_w, tile_h), batch) of the fastest candidate and the table
    {"WxH/B": median ms} (for the finalists, the median of the second pass)."""
    if key and cache_path:
        hit = _load(cache_path).get(key)
        if hit:
            return (tuple(hit["tile"]), int(hit["batch"])), hit.get("table")
    stream = torch.cuda.current_stream()
    table = {}
    for tile in tiles:
        for b in batches:
            if tile[0] * tile[1] == 512 and b > 64:
                continue  # not a valid tiling (at most 64 records per stage with 512-pixel tiles)
            set_tiling(tuple(tile), int(b))
            for _ in range(warmup):
                run()
            ms = float(np.median([_time(run, stream) for _ in range(reps)]))
            table[f"{tile[0]}x{tile[1]}/{b}"] = ms
    top = sorted(table, key=table.get)[:max(1, finalists)]
    if len(top) > 1:
        times = {k: [] for k in top}
        for _ in range(final_rounds):
            for k in top:
                (tw, th), b = k.split("/")[0].split("x"), k.split("/")[1]
                set_tiling((int(tw), int(th)), int(b))
                run()
                times[k] += [_time(run, stream) for _ in range(reps)]
        for k in top:
            table[k] = float(np.median(times[k]))
    name = min(top, key=table.get)
    (tw, th), b = name.split("/")[0].split("x"), name.split("/")[1]
    best = ((int(tw), int(th)), int(b))
    table = {k: round(v, 4) for k, v in table.items()}
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
