"""Launch-shape, chunk and batch-split autotuner for gsm_match_batch.

Searches, in two passes, workgroup size, pairs per lane per tile and the
first-level pair count above which a query gets launches of its own; then, on
the best of those, the LDS bytes a launch may use to stage rows and the
memory budget (which sets the chunk size of every level).  Every candidate
must reproduce the reference counts exactly (a candidate that disagrees is a
bug and raises); the fastest is cached per (device, graph size, query mix,
budget) in a JSON file so later runs reuse it without measuring.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import gsm

DEFAULT_SPACE = {
    "wg_size": [256, 512],
    "tile_items": [2, 4],
    "batch_heavy_pairs": [1 << 12, 1 << 16, 1 << 18, 1 << 20, 2 ** 64 - 1],
    # second pass, on the best of the first
    "stage_bytes": [16 << 10, 32 << 10, 48 << 10, 64 << 10],
    "budget_div": [1, 8],
}


def _key(graph: gsm.Graph, queries: Sequence, device: str, budget: int) -> str:
    info = graph.info()
    h = hashlib.sha1()
    for q in queries:
        h.update(np.asarray(q.edges, np.int32).tobytes())
        h.update(np.asarray(q.labels if q.labels is not None else [], np.int32).tobytes())
    return "%s|n=%d|nnz=%d|nq=%d|budget=%d|%s" % (device, info["n"], info["nnz"], len(queries), budget,
                                                  h.hexdigest()[:16])


def _time(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps


def tune_batch(graph: gsm.Graph, Qs: List[gsm.Query], workload_queries: Sequence, budget: int,
               cache_path: Optional[str] = None, space: Optional[Dict] = None, reps: int = 1,
               log=print) -> Dict:
    """Best {wg_size, tile_items, batch_heavy_pairs, stage_bytes, budget} for
    this batch (cached); pass the result's entries to gsm.match_batch."""
    import torch
    device = torch.cuda.get_device_name(0)
    key = _key(graph, workload_queries, device, budget)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        cache = json.load(open(cache_path))
        if key in cache:
            return cache[key]["best"]
    space = {**DEFAULT_SPACE, **(space or {})}
    ref = gsm.match_batch(graph, Qs, budget=budget)
    results = []

    def measure(cfg):
        got = gsm.match_batch(graph, Qs, **cfg)
        if not np.array_equal(got, ref):
            raise RuntimeError("autotune candidate %s changed the counts" % cfg)
        t = _time(lambda: gsm.match_batch(graph, Qs, **cfg), reps)
        results.append((t, cfg))
        log("autotune %s: %.1f ms" % (cfg, t * 1e3))
        return t

    # pass 1: launch shape and split at the default staging and the full budget
    first = []
    for wg in space["wg_size"]:
        for items in space["tile_items"]:
            for heavy in space["batch_heavy_pairs"]:
                cfg = {"wg_size": wg, "tile_items": items, "batch_heavy_pairs": heavy, "stage_bytes": 0,
                       "budget": budget}
                first.append((measure(cfg), cfg))
    base = min(first, key=lambda r: r[0])[1]
    # pass 2: staging bytes and chunk size (budget) on the best shape
    for stage in space["stage_bytes"]:
        for div in space["budget_div"]:
            cfg = dict(base, stage_bytes=stage, budget=max(budget // div, 1))
            if cfg == base:
                continue
            try:
                measure(cfg)
            except gsm.GsmError as e:
                if e.status != 5:  # a budget too small for these queries is skipped
                    raise
    results.sort(key=lambda r: r[0])
    best = results[0][1]
    if cache_path:
        cache[key] = {"best": best, "ms": round(results[0][0] * 1e3, 3),
                      "tried": [{"ms": round(t * 1e3, 3), **c} for t, c in results]}
        tmp = cache_path + ".tmp"
        json.dump(cache, open(tmp, "w"), indent=1)
        os.replace(tmp, cache_path)
    return best
