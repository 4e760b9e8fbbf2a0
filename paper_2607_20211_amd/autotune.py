"""Autotuner for the update path's launch schedule.

An update replays a captured HIP graph that queues a fixed number of hooking
rounds and super-forest search levels; batches that need more finish on the
host (extra launches and synchronisations), batches that need fewer pay for
launches that find nothing to do.  Which split is cheapest depends on the
workload (batch size, graph shape, how many graphs share a context), so it
is measured: every candidate (rounds queued, levels queued, delete scan mode)
replays the same sample updates from the same snapshot, and the fastest is
kept and cached on disk under a key describing the workload.  Results never
depend on the choice (tests check bit-exact results for every setting).
"""
from __future__ import annotations

import json
import os
import time

CANDIDATES = [(r, l, m) for r in (2, 3, 4, 6) for l in (2, 4, 6) for m in (0, 1)]


def cache_path() -> str:
    return os.environ.get("DRSF_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "drsf", "tune.json")


def _load_cache(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store_cache(path, cache):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only costs re-tuning


def tune(forest, sample, key: str, *, candidates=CANDIDATES, repeats: int = 2,
         use_cache: bool = True, sync=None) -> dict:
    """Pick the tunables for `forest` (a Forest or MultiForest).

    sample: callable(forest) that applies the sample updates (it runs from
    the same snapshot for every candidate); sync: callable that waits for the
    device (defaults to none: every apply already waits for its result).
    Returns {"rounds_queued", "levels_queued", "sweep_mode", "ms", "cached",
    "tried"} and leaves the best setting active and the state as it was."""
    path = cache_path()
    cache = _load_cache(path) if use_cache else {}
    if use_cache and key in cache:
        best = cache[key]
        forest.set_tuning(best["rounds_queued"], best["levels_queued"], best["sweep_mode"])
        return dict(best, cached=True, tried=0)
    snap = forest.snapshot()
    results = []
    try:
        for r, l, m in candidates:
            forest.set_tuning(r, l, m)
            t_best = None
            for _ in range(repeats):
                forest.restore(snap)
                if sync:
                    sync()
                t0 = time.perf_counter()
                sample(forest)
                if sync:
                    sync()
                t = time.perf_counter() - t0
                t_best = t if t_best is None else min(t_best, t)
            results.append((t_best, r, l, m))
        forest.restore(snap)
    finally:
        from .drsf import drsf_snapshot_free
        drsf_snapshot_free(snap)
    t, r, l, m = min(results)
    best = {"rounds_queued": r, "levels_queued": l, "sweep_mode": m, "ms": round(t * 1e3, 4)}
    forest.set_tuning(r, l, m)
    if use_cache:
        cache[key] = best
        _store_cache(path, cache)
    return dict(best, cached=False, tried=len(results))
