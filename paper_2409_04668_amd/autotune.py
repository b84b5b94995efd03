"""Autotuner: picks the schedule and launch shape by timing short pilot runs.

Single problems: history-based vs event-based schedule, persistent-grid
occupancy target (waves per CU) and, for event mode, the chunk of resident
histories.  Batched problems: work-queue chunk size and occupancy.  Results are
cached in a JSON file keyed by a hash of the problem data and the device name,
so a later run of the same workload skips the search.

Every candidate produces identical per-history results (the schedule never
changes a trajectory), so the tuner only trades speed.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import mcdc

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mcdc_mi355x_autotune.json")


def _hash_problem(prob) -> str:
    h = hashlib.sha256()

    def feed(x):
        if isinstance(x, dict):
            for k in sorted(x):
                h.update(k.encode())
                feed(x[k])
        elif isinstance(x, (list, tuple)):
            for v in x:
                feed(v)
        elif isinstance(x, np.ndarray):
            h.update(np.ascontiguousarray(x).tobytes())
        else:
            h.update(repr(x).encode())

    feed(prob)
    return h.hexdigest()[:20]


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path, data):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_single(prob, opt, n, seed) -> float:
    import torch
    gp = mcdc.Problem(prob, opt)
    gp.run(min(n, 200_000), seed)            # warm-up (code objects, caches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gp.run(n, seed + 1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gp.close()
    return n / dt


def tune_single(prob, pilot=2_000_000, waves=(8, 12, 16, 24, 32), event_chunks=(1 << 20, 1 << 22),
                cache_path=DEFAULT_CACHE, use_cache=True, seed=12345):
    """Returns {"options": dict for mcdc.make_options, "histories_per_s": ..., "trials": [...]}."""
    key = "single:" + _device_name() + ":" + _hash_problem(prob) + f":{pilot}"
    cache = _load(cache_path) if use_cache else {}
    if key in cache:
        return cache[key]
    trials = []
    for w in waves:
        o = dict(schedule=mcdc.SCHED_HISTORY, waves_per_cu=w)
        trials.append((o, _time_single(prob, mcdc.make_options(**o), pilot, seed)))
    if prob.get("importance") is None:
        for ch in event_chunks:
            o = dict(schedule=mcdc.SCHED_EVENT, event_chunk=ch)
            trials.append((o, _time_single(prob, mcdc.make_options(**o), pilot, seed)))
    best = max(trials, key=lambda t: t[1])
    res = {"options": best[0], "histories_per_s": best[1],
           "trials": [{"options": o, "histories_per_s": r} for o, r in trials]}
    if use_cache:
        cache[key] = res
        _save(cache_path, cache)
    return res


def tune_batch(probs, n_hist, chunks=(512, 2048, 8192), waves=(8, 16), cache_path=DEFAULT_CACHE,
               use_cache=True, seed=777):
    """Chunk size and occupancy of the batched persistent kernel."""
    import torch
    key = "batch:" + _device_name() + ":" + _hash_problem([probs, np.asarray(n_hist)])
    cache = _load(cache_path) if use_cache else {}
    if key in cache:
        return cache[key]
    total = float(np.sum(n_hist))
    trials = []
    for ch in chunks:
        for w in waves:
            o = dict(event_chunk=ch, waves_per_cu=w)
            bp = mcdc.BatchProblem(probs, n_hist, mcdc.make_options(**o))
            bp.run(seed)                     # warm-up + graph capture
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bp.run(seed + 1)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            bp.close()
            trials.append((o, total / dt))
    best = max(trials, key=lambda t: t[1])
    res = {"options": best[0], "histories_per_s": best[1],
           "trials": [{"options": o, "histories_per_s": r} for o, r in trials]}
    if use_cache:
        cache[key] = res
        _save(cache_path, cache)
    return res
