"""Autotuner for the update path's launch schedule.

An update launches a fixed kernel sequence (kernel by kernel, or as a
captured HIP graph) that queues a fixed number of hooking rounds and
super-forest search levels; batches that need more finish on the
host (extra launches and synchronisations), batches that need fewer pay for
launches that find nothing to do.  Which split is cheapest depends on the
workload (batch size, graph shape, how many graphs share a context), so it
is measured: every candidate (rounds queued, levels queued, delete scan mode)
replays the same sample updates from the same snapshot, and the fastest is
kept and cached on disk under a key describing the workload.  Results never
depend on the choice (tests check bit-exact results for every setting).

For the batched pattern (multi-graph contexts) tune_batched also searches
the small-graph engine: the LDS threshold (graphs of at most that many
vertices are updated whole by one workgroup each; a threshold needs its own
context, since it decides where each graph's edges live), then the
engine's workgroup size and number of persistent workgroups on the best
threshold's context, then the schedule above.
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


THRESHOLDS = (0, 1024, 2048, 4096, 8192)
SMALL_SCHEDULES = [(t, w) for t in (256, 512, 1024) for w in (0, 128, 512)]


def _time(forest, snap, sample, repeats, sync):
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
    forest.restore(snap)
    return t_best


def tune_batched(make, sample, key: str, *, thresholds=THRESHOLDS, small_schedules=SMALL_SCHEDULES,
                 candidates=CANDIDATES, repeats: int = 2, sync=None):
    """Pick the batched pattern's schedule.  make(threshold) builds a
    MultiForest with that small_graph_vertices; sample(forest) applies the
    sample updates.  Returns (forest, choice): the best threshold's context,
    left with the best small-graph schedule and launch schedule active and
    its state as created, and {"small_graph_vertices", "small_threads",
    "small_workgroups", "rounds_queued", "levels_queued", "sweep_mode",
    "ms", "tried"}."""
    from .drsf import drsf_snapshot_free
    best_t, best_f, best_ms, tried = None, None, None, 0
    per_threshold = {}
    for th in thresholds:
        f = make(th)
        snap = f.snapshot()
        try:
            t = _time(f, snap, sample, repeats, sync)
        finally:
            drsf_snapshot_free(snap)
        per_threshold[th] = round(t * 1e3, 4)
        tried += 1
        if best_ms is None or t < best_ms:
            if best_f is not None:
                best_f.close()
            best_t, best_f, best_ms = th, f, t
        else:
            f.close()
    f = best_f
    snap = f.snapshot()
    sched = (0, 0)
    try:
        if best_t:
            res = []
            for th, wg in small_schedules:
                f.set_small_schedule(th, wg)
                res.append((_time(f, snap, sample, repeats, sync), th, wg))
                tried += 1
            t, th, wg = min(res)
            sched = (th, wg)
            f.set_small_schedule(th, wg)
    finally:
        drsf_snapshot_free(snap)
    inner = tune(f, sample, key, candidates=candidates, repeats=repeats, use_cache=False, sync=sync)
    choice = {"small_graph_vertices": best_t, "small_threads": sched[0] or 512,
              "small_workgroups": sched[1], "rounds_queued": inner["rounds_queued"],
              "levels_queued": inner["levels_queued"], "sweep_mode": inner["sweep_mode"],
              "ms": inner["ms"], "tried": tried + inner["tried"],
              "threshold_ms": per_threshold}
    return f, choice
