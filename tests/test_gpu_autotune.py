"""The batch autotuner: every candidate it measures, and the configuration
it picks, gives the same counts as the defaults (it raises otherwise), the
picked one is reused from the cache without measuring, and a cache keyed on
another budget is not."""
import json

import numpy as np
import pytest

from paper_2003_01527_amd import autotune, gsm
from paper_2003_01527_amd import workloads as W

pytestmark = pytest.mark.gpu

SPACE = {"wg_size": [256, 512], "tile_items": [2, 4], "batch_heavy_pairs": [1 << 16, (1 << 64) - 1],
         "stage_bytes": [16 << 10, 64 << 10], "budget_div": [1, 4]}


def test_tuned_counts_equal_defaults_and_cache_is_reused(tmp_path, monkeypatch):
    w = W.batch(nq=64, cap=float(2 ** 24))
    G = gsm.Graph.from_workload(w.graph)
    Qs = [gsm.Query.from_workload(q) for q in w.queries]
    budget = 1 << 30
    cache = str(tmp_path / "tune.json")
    best = autotune.tune_batch(G, Qs, w.queries, budget, cache_path=cache, space=SPACE, log=lambda *a: None)
    assert set(best) == {"wg_size", "tile_items", "batch_heavy_pairs", "stage_bytes", "budget"}
    ref = gsm.match_batch(G, Qs, budget=budget)
    np.testing.assert_array_equal(gsm.match_batch(G, Qs, **best), ref)
    # single-query matching with the tuned launch shape gives the same counts
    per = [gsm.match(G, Q, wg_size=best["wg_size"], tile_items=best["tile_items"],
                     stage_bytes=best["stage_bytes"], budget=best["budget"])[0] for Q in Qs]
    np.testing.assert_array_equal(np.array(per, np.uint64), ref)
    tried = json.load(open(cache))
    assert len(tried) == 1 and len(next(iter(tried.values()))["tried"]) >= 8
    # the second call reads the cache and launches nothing
    calls = []
    monkeypatch.setattr(gsm, "match_batch", lambda *a, **k: calls.append(1))
    again = autotune.tune_batch(G, Qs, w.queries, budget, cache_path=cache, space=SPACE)
    assert again == best and not calls
    # another budget is another key
    monkeypatch.undo()
    other = autotune.tune_batch(G, Qs, w.queries, budget // 2, cache_path=cache,
                                space=dict(SPACE, wg_size=[256], tile_items=[4]), log=lambda *a: None)
    assert len(json.load(open(cache))) == 2
    np.testing.assert_array_equal(gsm.match_batch(G, Qs, **other), ref)
