"""Autotuner: picks the schedule and launch shape by timing short pilot runs.

Single problems: history-based, event-based or hybrid schedule,
persistent-grid occupancy target (waves per CU) and, for the event and hybrid
schedules, the chunk of resident histories.  The k-eigenvalue mode: the
history kernel's occupancy for the generation size, with or without a hot
tile.  Batched problems: work-queue chunk size and occupancy.  Results are
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


def tune_single(prob, pilot=2_000_000, waves=(8, 12, 16, 24, 32),
                event_chunks=(1 << 20, 1 << 22, 1 << 23), tile=None, cache_path=DEFAULT_CACHE,
                use_cache=True, seed=12345, schedules=None):
    """Returns {"options": dict for mcdc.make_options, "histories_per_s": ..., "trials": [...]}.
    Tries the history schedule at each occupancy and the event and hybrid
    schedules at each chunk size (`schedules` restricts the set).  `tile` =
    (lo[5], n[5]), e.g. from plan_hot_tile: the LDS hot tile of the history
    schedule, of the hybrid schedule's lead and re-lead stages and of the
    event schedule's flight stage.  Population control runs
    only in the event and hybrid schedules, with every batch of the pilot
    resident (chunks below the batch size are skipped)."""
    tj = None if tile is None else [[int(v) for v in tile[0]], [int(v) for v in tile[1]]]
    allowed = set(schedules or (mcdc.SCHED_HISTORY, mcdc.SCHED_EVENT, mcdc.SCHED_HYBRID))
    key = ("single:" + _device_name() + ":" + _hash_problem(prob) + f":{pilot}:{tj}:" +
           ",".join(str(v) for v in sorted(allowed)))
    cache = _load(cache_path) if use_cache else {}
    if key in cache:
        return cache[key]
    trials = []
    pc = prob.get("population_control") is not None

    def trial(**o):
        if tj is not None:
            o["tile"] = tj
        trials.append((o, _time_single(prob, mcdc.make_options(**o), pilot, seed)))

    if not pc and mcdc.SCHED_HISTORY in allowed:
        for w in waves:
            trial(schedule=mcdc.SCHED_HISTORY, waves_per_cu=w)
    if prob.get("importance") is None:
        batch = -(-pilot // int(prob["n_batches"]))
        for ch in event_chunks:
            if pc and ch < batch:
                continue
            for sched in (mcdc.SCHED_EVENT, mcdc.SCHED_HYBRID):
                if sched in allowed:
                    trial(schedule=sched, event_chunk=ch)
    if not trials:
        raise ValueError("no schedule can run this problem at this pilot size")
    best = max(trials, key=lambda t: t[1])
    res = {"options": best[0], "histories_per_s": best[1],
           "trials": [{"options": o, "histories_per_s": r} for o, r in trials]}
    if use_cache:
        cache[key] = res
        _save(cache_path, cache)
    return res


def grow_tile(density: np.ndarray, max_bins: int):
    """Box over a 5-D density [g][t][z][y][x] (any non-negative weights) of at
    most max_bins bins: start at the densest bin and repeatedly add the face
    slab (10 candidates) with the largest mass per added bin.  Returns
    (lo, n) in x, y, z, t, g order and the captured fraction."""
    D = np.asarray(density, float)
    total = D.sum()
    idx = np.unravel_index(int(np.argmax(D)), D.shape)
    lo = list(idx)
    hi = [i + 1 for i in idx]
    vol = 1
    while True:
        best = None
        for ax in range(5):
            ext = hi[ax] - lo[ax]
            add = vol // ext
            if vol + add > max_bins:
                continue
            for side in (0, 1):
                k = lo[ax] - 1 if side == 0 else hi[ax]
                if k < 0 or k >= D.shape[ax]:
                    continue
                sl = [slice(lo[a], hi[a]) for a in range(5)]
                sl[ax] = slice(k, k + 1)
                gain = D[tuple(sl)].sum() / add
                if best is None or gain > best[0]:
                    best = (gain, ax, side, add)
        if best is None or best[0] <= 0.0:
            break
        _, ax, side, add = best
        if side == 0:
            lo[ax] -= 1
        else:
            hi[ax] += 1
        vol += add
    frac = D[tuple(slice(lo[a], hi[a]) for a in range(5))].sum() / total if total > 0 else 0.0
    # density axes are (g, t, z, y, x); options want (x, y, z, t, g)
    order = [4, 3, 2, 1, 0]
    return ([lo[a] for a in order], [hi[a] - lo[a] for a in order]), float(frac)


def plan_hot_tile(prob, pilot=2_000_000, max_bins=None, seed=4242):
    """Pilot run -> LDS hot tile over the bins with the most track length.
    Returns (tile, captured fraction) or (None, 0) when the whole mesh fits
    the ordinary LDS tile anyway."""
    max_bins = max_bins or mcdc.MAX_TILE_BINS
    from . import workloads as W
    nb = W.n_bins(prob)
    if nb <= 7680:
        return None, 0.0
    q = W.with_(prob, n_batches=1, ww=None, importance=None)
    gp = mcdc.Problem(q, mcdc.make_options(mcdc.SCHED_HISTORY))
    gp.run(pilot, seed)
    s, _ = gp.raw()
    gp.close()
    m = prob["mesh"]
    nx, ny, nz, nt = [int(v) for v in m["n"]]
    G = prob["sigma_t"].shape[1] if m["per_group"] else 1
    return grow_tile(s.reshape(G, nt, nz, ny, nx), max_bins)


def plan_keff_tile(prob, m=200_000, generations=5, max_bins=None, seed=4243):
    """plan_hot_tile for a problem with fission, whose pilot is a few
    k-eigenvalue generations of m histories (a fixed-source run refuses a
    fissile problem).  Returns (tile, captured fraction) or (None, 0)."""
    max_bins = max_bins or mcdc.MAX_TILE_BINS
    from . import workloads as W
    if W.n_bins(prob) <= 7680:
        return None, 0.0
    gp = mcdc.Problem(W.with_(prob, n_batches=1), mcdc.make_options(mcdc.SCHED_HISTORY))
    gp.run_keff(m, generations - 1, 1, seed=seed)
    s, _ = gp.raw()
    gp.close()
    mm = prob["mesh"]
    nx, ny, nz, nt = [int(v) for v in mm["n"]]
    G = prob["sigma_t"].shape[1] if mm["per_group"] else 1
    return grow_tile(np.asarray(s).reshape(G, nt, nz, ny, nx), max_bins)


def _time_keff(prob, opt, m, generations, seed) -> float:
    import torch
    n_in, n_act = generations
    gp = mcdc.Problem(prob, opt)
    gp.run_keff(min(m, 100_000), 1, 1, seed=seed)        # warm-up
    gp.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gp.run_keff(m, n_in, n_act, seed=seed + 1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gp.close()
    return m * (n_in + n_act) / dt


def tune_keff(prob, m, waves=(4, 8, 16), tile=None, generations=(1, 2), cache_path=DEFAULT_CACHE,
              use_cache=True, seed=2468):
    """Occupancy (waves per CU) of the k-eigenvalue mode's history kernel
    for generations of m histories, and whether the LDS hot tile `tile`
    (e.g. from plan_keff_tile) pays: a generation is one launch, so with few
    histories per work-item the grid size matters.  Each candidate runs a
    warm-up, then `generations` = (inactive, active) generations of m
    histories, timed.  Every candidate gives the same trajectories."""
    tj = None if tile is None else [[int(v) for v in tile[0]], [int(v) for v in tile[1]]]
    key = "keff:" + _device_name() + ":" + _hash_problem(prob) + f":{m}:{tj}:{tuple(waves)}"
    cache = _load(cache_path) if use_cache else {}
    if key in cache:
        return cache[key]
    trials = []

    def trial(**o):
        o = dict(schedule=mcdc.SCHED_HISTORY, **o)
        trials.append((o, _time_keff(prob, mcdc.make_options(**o), m, generations, seed)))

    for w in waves:
        trial(waves_per_cu=w)
    if tj is not None:
        trial(tile=tj)
    best = max(trials, key=lambda t: t[1])
    res = {"options": best[0], "histories_per_s": best[1],
           "trials": [{"options": o, "histories_per_s": r} for o, r in trials]}
    if use_cache:
        cache[key] = res
        _save(cache_path, cache)
    return res


def tune_batch(probs, n_hist, chunks=(2048, 8192, 16384), waves=(8, 16), cache_path=DEFAULT_CACHE,
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
