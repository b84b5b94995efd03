"""Benchmark: histories/s of the analog time-dependent transport loop on the
3D duct problem (60x100x60 cm box, bent 10x10 cm void duct, 1 cm mesh x 20
time bins = 7.2e6 FP64 bins, 1e8 histories per step) on one MI355X.

One step = one mcdc_run of 1e8 source histories (20 batches) under the
schedule the autotuner picks, with all inputs resident in HBM.  Prints one
JSON line with:
  * the roofline of the tracking kernel.  Its binding limit is VALU issue
    under divergence, so the headline is the ALU roofline: useful VALU
    lane-instructions per launch (SQ counters of the committed profile) over
    the launch time measured here, against 256 CUs x 4 SIMDs x 16 lanes x
    2.4 GHz.  Beside it the memory views: HBM bytes (16 B per FP64 atomic
    update that reaches HBM, the HBM share of the updates taken from the
    committed PMC write requests) against 8 TB/s and the measured copy rate,
    HBM atomics against the measured random-atomic ceiling, LDS ds_add_f64
    updates against the measured LDS ceiling;
  * the figure of merit 1/(R^2 T) at 1% detector relative error of the
    analog run against the learned weight windows (window map, and the
    network evaluated at every check), measured after the timed steps;
  * the 256-problem batched workload's rate;
  * the CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_PIECE = 16.0          # FP64 atomic read-modify-write: 8 B read + 8 B written
# VALU issue peak: 256 CUs x 4 SIMDs, each retiring a wave64 instruction every
# 4 cycles (16 lanes per cycle), at 2.4 GHz
VALU_LANE_PEAK = 256 * 4 * 16 * 2.4e9
ATOMIC_REQUEST_BYTES = 32.0     # one device-scope FP64 atomic = one 32-byte write request
KERNEL_SOURCES = ["transport_device.hpp", "transport_stages.hpp", "lane_stack.hpp",
                  "mcdc_internal.hpp", "mcdc_history.hip", "mcdc_event.hip"]
SCHED_NAMES = {1: "history", 2: "event", 3: "hybrid"}
# the tracking kernel whose launches are timed under each schedule
TIMED_KERNEL = {1: "k_history", 2: "k_ev_flight", 3: "k_ev_lead"}


def pmc_summary(kernel: str) -> str:
    return os.path.join(ROOT, "profiles", f"{kernel}_duct_1e8_pmc.txt")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2409_04668_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, histories_per_launch: float):
    """HBM bytes per launch of `kernel` from its committed rocprofv3 PMC
    summary, or None if there is none, the kernels changed since, or its
    launches held another number of histories."""
    path = pmc_summary(kernel)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_sha") != kernel_hash():
        return None
    try:
        h = float(vals["histories_per_launch"])
    except (KeyError, ValueError):
        return None
    if abs(h - histories_per_launch) > 1e-3 * histories_per_launch:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measured_valu(kernel: str):
    """VALU issue figures of `kernel` from its committed SQ-counter summary
    (None if there is none or the kernels changed since)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_duct_1e8_sq.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_sha") != kernel_hash():
        return None
    try:
        return {"simd_valu_busy_fraction": float(vals["simd_valu_busy_fraction"]),
                "active_lanes_per_valu_instruction": float(vals["active_lanes_per_valu_instruction"].split()[0]),
                "lane_throughput_fraction": float(vals["lane_throughput_fraction"]),
                "lane_instructions_per_launch": float(vals["SQ_THREAD_CYCLES_VALU"]),
                "histories_per_launch": float(vals.get("histories_per_launch", "nan")),
                "source": os.path.relpath(path, ROOT)}
    except (KeyError, ValueError):
        return None


def roofline(kernel, launches, avg_launch_s, hist_per_launch, pieces_per_launch, traffic,
             ceil_rand, ceil_run8, ceil_lds, copy_bw):
    """The tracking kernel's roofline object.  Every rate divides per-launch
    work by the mean launch time measured in this run (HIP events on the
    launch stream).  Work per launch: VALU lane-instructions from the
    committed SQ summary (scaled to this run's histories per launch); scored
    pieces from the run's own counters, split into HBM updates (PMC write
    requests of the committed summary, 32 B each, which also count the tile
    flushes: an upper bound) and LDS updates (the rest)."""
    out = {"kernel": kernel, "launches": launches, "avg_launch_ms": 1e3 * avg_launch_s,
           "histories_per_launch": hist_per_launch, "traffic": traffic}
    # memory side
    if traffic is not None:
        hbm_updates = min(traffic / ATOMIC_REQUEST_BYTES, pieces_per_launch)
        share = "measured (PMC WRITE_SIZE / 32 B)"
    else:
        hbm_updates = pieces_per_launch
        share = "unknown (no current PMC summary): every piece counted as an HBM update"
    lds_updates = pieces_per_launch - hbm_updates
    hbm_bytes = BYTES_PER_PIECE * hbm_updates
    hbm_gbps = hbm_bytes / avg_launch_s / 1e9
    hbm_rate = hbm_updates / avg_launch_s
    lds_rate = lds_updates / avg_launch_s
    out["hbm"] = {"algorithmic_bytes_per_launch": hbm_bytes, "achieved_GBps": hbm_gbps,
                  "peak_GBps": HBM_PEAK_GBS, "frac_of_peak": hbm_gbps / HBM_PEAK_GBS,
                  "measured_copy_GBps": copy_bw / 1e9,
                  "frac_of_measured": hbm_gbps / (copy_bw / 1e9) if copy_bw else None}
    out["atomics"] = {"pieces_per_launch": pieces_per_launch,
                      "hbm_updates_per_launch": hbm_updates, "lds_updates_per_launch": lds_updates,
                      "hbm_share": share,
                      "hbm_updates_per_s": hbm_rate,
                      "hbm_frac_of_random_ceiling": hbm_rate / ceil_rand if ceil_rand else None,
                      "hbm_frac_of_runs8_ceiling": hbm_rate / ceil_run8 if ceil_run8 else None,
                      "lds_updates_per_s": lds_rate,
                      "lds_frac_of_ceiling": lds_rate / ceil_lds if ceil_lds else None}
    mem = [f for f in (out["hbm"]["frac_of_measured"], out["atomics"]["hbm_frac_of_random_ceiling"])
           if f is not None]
    out["memory_frac"] = max(mem) if mem else None     # max(HBM, atomic) against measured ceilings
    # ALU side: the binding limit
    valu = measured_valu(kernel)
    out["valu_issue"] = valu
    if valu is not None and valu["histories_per_launch"] > 0:
        lanes = valu["lane_instructions_per_launch"] * hist_per_launch / valu["histories_per_launch"]
        ach = lanes / avg_launch_s
        out.update(bound="alu", achieved=ach / 1e12, peak=VALU_LANE_PEAK / 1e12,
                   unit="T VALU lane-instructions/s", frac=ach / VALU_LANE_PEAK,
                   lane_instructions_per_launch=lanes)
    else:
        out.update(bound="hbm", achieved=hbm_gbps, peak=HBM_PEAK_GBS, unit="GB/s",
                   frac=hbm_gbps / HBM_PEAK_GBS)
    return out


def cpu_baseline(prob, n_sample, seed):
    from oracle import oracle as O
    O.build(force=False)
    r = O.OracleRun(prob)
    r.run(n_sample, seed)
    return dict(value=n_sample / r.last_seconds, unit="histories/s", cores=1, kind="oracle",
                sample=f"{n_sample} histories of the same duct problem, single-threaded C oracle, "
                       f"{r.last_seconds:.1f} s")


def duct_options(args, mcdc, prob):
    """Options of the duct runs: the LDS hot tile placed from a short analog
    pilot, then (--schedule auto) the schedule the autotuner picks from
    2e7-history trials of the history, event and hybrid schedules.  Setup,
    not timed.  Returns (options dict, tuner result or None, tile, captured
    fraction)."""
    from paper_2409_04668_amd import autotune
    tile, tile_frac = (None, 0.0) if args.no_tile else autotune.plan_hot_tile(prob, pilot=1_000_000)
    tuned = None
    if args.schedule == "auto":
        tuned = autotune.tune_single(prob, pilot=20_000_000, waves=(16,), event_chunks=(1 << 25,),
                                     tile=tile, use_cache=False)
        oargs = dict(tuned["options"])
    else:
        sched = {"history": mcdc.SCHED_HISTORY, "event": mcdc.SCHED_EVENT,
                 "hybrid": mcdc.SCHED_HYBRID}[args.schedule]
        oargs = dict(schedule=sched, event_chunk=1 << 25)
        if tile is not None:
            oargs["tile"] = [[int(v) for v in tile[0]], [int(v) for v in tile[1]]]
    if args.waves_per_cu:
        oargs["waves_per_cu"] = args.waves_per_cu
    return oargs, tuned, tile, tile_frac


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--histories", type=int, default=100_000_000)
    ap.add_argument("--schedule", choices=["auto", "history", "event", "hybrid"], default="auto")
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=20_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fom", action="store_true",
                    help="skip the analog vs learned-weight-window FOM comparison")
    ap.add_argument("--no-other-schedule", action="store_true",
                    help="skip the comparison step under the other schedule")
    ap.add_argument("--no-tile", action="store_true", help="tally straight to HBM atomics")
    ap.add_argument("--workload", choices=["duct", "batch", "fom"], default="duct")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES (PMC calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(histories would shard by history-id range across GPUs, with one sum of the "
              "batch tallies)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2409_04668_amd import mcdc
    from paper_2409_04668_amd import workloads as W

    if args.calibrate_copy:
        n = args.calibrate_copy // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8, "copies": 3}), flush=True)
        return
    if args.workload == "batch":
        return bench_batch(args, torch, mcdc, W)
    if args.workload == "fom":
        return bench_fom(args, torch, mcdc, W)

    prob = W.config2()
    oargs, tuned, tile, tile_frac = duct_options(args, mcdc, prob)
    sched = oargs["schedule"]
    kernel = TIMED_KERNEL[sched]
    gp = mcdc.Problem(prob, mcdc.make_options(**oargs))
    N = args.histories
    seed = 20260001
    for i in range(args.warmup):
        gp.run(N, seed + i)
    torch.cuda.synchronize()
    c0 = gp.counters()
    gp.kernel_time()                       # drop warm-up launches
    gp.set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        gp.run(N, seed + args.warmup + i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gp.set_kernel_timing(False)
    launches, kms = gp.kernel_time()
    c1 = gp.counters()
    T = t1 - t0
    n_done = args.steps * N
    pieces = c1["pieces"] - c0["pieces"]
    avg_launch_s = kms / 1e3 / max(launches, 1)
    hist_per_launch = n_done / max(launches, 1)
    pieces_per_launch = pieces / max(launches, 1)
    traffic = measured_traffic(kernel, hist_per_launch)
    det_mean, det_rel = gp.tallies(mcdc.TALLY_DETECTOR)
    # measured ceilings: FP64 atomics scattered over an array of the tally's
    # size (fully random, and in runs of 8 consecutive bins like the mesh
    # walk), LDS ds_add_f64 into an array of the hot tile's size per
    # workgroup, and a streaming copy
    nb = W.n_bins(prob)
    ceil_rand = mcdc.micro_atomic_rate(nb, int(pieces_per_launch), run=1)
    ceil_run8 = mcdc.micro_atomic_rate(nb, int(pieces_per_launch), run=8)
    tile_bins = int(np.prod(tile[1])) if tile is not None else 7680
    ceil_lds = mcdc.micro_lds_atomic_rate(tile_bins, 2_000_000_000)
    copy_bw = mcdc.micro_copy_rate()
    roof = roofline(kernel, launches, avg_launch_s, hist_per_launch, pieces_per_launch, traffic,
                    ceil_rand, ceil_run8, ceil_lds, copy_bw)
    out = {
        "metric": "histories/s (analog, FP64 tallies) on the 3D duct problem",
        "value": n_done / T,
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D duct 60x100x60 cm, 1 group, 1 cm mesh x 20 t-bins "
                               "(7.2e6 FP64 bins), analog, 1e8 histories per step",
                   "histories_per_step": N, "schedule": SCHED_NAMES[sched],
                   "options": oargs,
                   "autotune_trials": tuned["trials"] if tuned else None,
                   "tally_bins": W.n_bins(prob),
                   "lds_hot_tile": None if tile is None else
                   {"lo_xyztg": [int(v) for v in tile[0]], "n_xyztg": [int(v) for v in tile[1]],
                    "pilot_track_length_fraction": tile_frac}},
        "roofline": roof,
        "pieces_per_history": pieces / n_done,
        "flights_per_history": (c1["flights"] - c0["flights"]) / n_done,
        "detector": {"mean": float(det_mean[0]), "rel_err": float(det_rel[0])},
    }
    out["measured_ceilings"] = {
        "fp64_atomics_random_per_s": ceil_rand, "fp64_atomics_runs8_per_s": ceil_run8,
        "lds_fp64_atomics_per_s": ceil_lds, "lds_ceiling_bins": tile_bins,
        "copy_GBps": copy_bw / 1e9}
    # the paper's own rate, quoted as context only (other problem, other GPU):
    # 1e10 histories of its time-dependent duct benchmark in 1500 s on one V100
    out["paper_context"] = {"histories_per_s": 1e10 / 1500.0, "hardware": "1x NVIDIA V100 (Lassen)",
                            "workload": "Kobayashi dog-leg void duct, time dependent, 1 group",
                            "source": "Sec. Performance (GPU profiling paragraph)"}
    gp.close()
    # the same step under the other schedules (with the tile),
    # one timed step after a warm-up, as a comparison
    if not args.no_other_schedule:
        out["other_schedules"] = {}
        for osched in (mcdc.SCHED_HISTORY, mcdc.SCHED_EVENT, mcdc.SCHED_HYBRID):
            if osched == sched:
                continue
            o = dict(schedule=osched, event_chunk=1 << 25)
            if tile is not None:
                o["tile"] = tile
            go = mcdc.Problem(prob, mcdc.make_options(**o))
            go.run(N, seed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            go.run(N, seed + 1)
            torch.cuda.synchronize()
            out["other_schedules"][SCHED_NAMES[osched]] = N / (time.perf_counter() - t0)
            go.close()
    if not args.no_other_schedule:
        # the same step with the collision estimator as a second mesh tally
        pc = dict(prob, collision_tally=True)
        gc = mcdc.Problem(pc, mcdc.make_options(**oargs))
        gc.run(N, seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gc.run(N, seed + 1)
        torch.cuda.synchronize()
        rate = N / (time.perf_counter() - t0)
        out["with_collision_estimator"] = {"histories_per_s": rate,
                                           "relative_to_track_length_only": rate / out["value"]}
        gc.close()
        # the same step with a surface-current tally on the plane y = 45 cm
        # (crossings of the first leg, binned on the x-z mesh and in time)
        ps = dict(prob, surface_tally=dict(axis=1, pos=45.0))
        gs = mcdc.Problem(ps, mcdc.make_options(**oargs))
        gs.run(N, seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gs.run(N, seed + 1)
        torch.cuda.synchronize()
        rate = N / (time.perf_counter() - t0)
        out["with_surface_current_tally"] = {"histories_per_s": rate,
                                             "relative_to_track_length_only": rate / out["value"],
                                             "crossings_per_history": gs.counters()["surf_crossings"] / (2 * N)}
        gs.close()
    if not args.no_other_schedule:
        # the 7-group duct (5.04e7 tally bins), hybrid schedule with its own
        # planned tile, one timed step of the same size after a warm-up
        from paper_2409_04668_amd import autotune
        p7 = W.config3()
        tile7, frac7 = autotune.plan_hot_tile(p7, pilot=1_000_000)
        g7 = mcdc.Problem(p7, mcdc.make_options(mcdc.SCHED_HYBRID, event_chunk=1 << 25,
                                                tile=tile7))
        g7.run(N, seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g7.run(N, seed + 1)
        torch.cuda.synchronize()
        out["multigroup_duct_7_groups"] = {
            "histories_per_s": N / (time.perf_counter() - t0), "tally_bins": W.n_bins(p7),
            "schedule": "hybrid", "tile_track_length_fraction": frac7,
            "flights_per_history": g7.counters()["flights"] / (2 * N)}
        g7.close()
    if not args.no_other_schedule:
        # population control at census: the duct problem with 20 census steps
        # under the hybrid schedule with the duct's hot tile, without and with
        # splitting-roulette to one particle per source history at every census
        rates = {}
        for name, target in (("without", None), ("with_target_1", 1.0)):
            pp = W.config2(n_census=20)
            if target is not None:
                pp["population_control"] = dict(target=target)
            # population control holds one batch of histories resident
            gq = mcdc.Problem(pp, mcdc.make_options(mcdc.SCHED_HYBRID, event_chunk=N // 20,
                                                    tile=tile))
            gq.run(N, seed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gq.run(N, seed + 1)
            torch.cuda.synchronize()
            rates[name] = N / (time.perf_counter() - t0)
            if target is not None:
                c = gq.counters()
                rates["pc_kills_per_history"] = c["pc_kills"] / (2 * N)
                rates["pc_copies_per_history"] = c["pc_copies"] / (2 * N)
            gq.close()
        out["population_control_hybrid_20_census"] = {
            "hot_tile": tile is not None,
            "histories_per_s_without": rates["without"],
            "histories_per_s_with": rates["with_target_1"],
            "pc_kills_per_history": rates["pc_kills_per_history"],
            "pc_copies_per_history": rates["pc_copies_per_history"]}
    if not args.no_other_schedule:
        out["batched_256_problems"] = batch_rate(torch, mcdc, W, steps=3, warmup=1)
        out["k_eigenvalue"] = keff_rate(torch, mcdc, W)
    if not args.no_fom:
        out["fom"] = fom_comparison(mcdc, W, oargs, tile)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_sample, seed)
    print(json.dumps(out), flush=True)


def batch_rate(torch, mcdc, W, steps, warmup):
    """256 batched problems (1e4-1e6 histories each, 10 census steps): one
    pass = every problem's histories, one persistent launch per census step,
    graph-replayed; work-chunk size and occupancy from the autotuner (full
    passes, setup).  Histories/s over the whole batch."""
    probs, n_hist = W.config5()
    from paper_2409_04668_amd import autotune
    tuned = autotune.tune_batch(probs, n_hist, use_cache=False)
    bp = mcdc.BatchProblem(probs, n_hist, mcdc.make_options(**tuned["options"]))
    total = int(n_hist.sum())
    for i in range(warmup):
        bp.run(7 + i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        bp.run(1000 + i)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    pieces = sum(bp.counters(p)["pieces"] for p in range(len(probs)))
    bp.close()
    return {"histories_per_s": total * steps / T, "ms_per_pass": 1e3 * T / steps,
            "passes": steps, "histories_per_pass": total,
            "workload": "256 box problems, 1-8 regions, 1-7 groups, 20^3 x 10 t-bins each",
            "autotuned_options": tuned["options"], "autotune_trials": tuned["trials"],
            "pieces_per_history": pieces / (total * (steps + warmup))}


def keff_rate(torch, mcdc, W, M=1_000_000, n_inactive=5, n_active=10):
    """The k-eigenvalue mode on the two-group reflected core (30^3 x 2 mesh
    bins), under the occupancy (and hot tile) the autotuner picks for
    generations of M histories: one warm-up iteration, then n_inactive +
    n_active generations of M histories timed; the mean of each estimator
    over the active generations with its standard error."""
    import numpy as np
    from paper_2409_04668_amd import autotune
    p = W.keff_core(nx=30)
    # the history kernel's occupancy for this generation size, and whether a
    # hot tile pays, from short runs (setup, not timed)
    tile, frac = autotune.plan_keff_tile(p)
    choice = autotune.tune_keff(p, M, tile=tile, use_cache=False)
    gp = mcdc.Problem(p, mcdc.make_options(**choice["options"]))
    gp.run_keff(100_000, 1, 2, seed=5)
    gp.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = gp.run_keff(M, n_inactive, n_active, seed=6)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    c = gp.counters()
    gp.close()

    def stats(k):
        k = np.asarray(k, float)[n_inactive:]
        return float(k.mean()), float(k.std(ddof=1) / np.sqrt(k.size))
    kc, sc = stats(out["k_col"])
    ks, ss = stats(out["k_site"])
    n = M * (n_inactive + n_active)
    return {"workload": "two-group reflected core (40 cm fissile cube in a 60 cm reflector), "
                        "30^3 x 2 mesh bins, history schedule",
            "autotuned_options": choice["options"], "autotune_trials": choice["trials"],
            "tile_track_length_fraction": frac,
            "histories_per_generation": M, "generations": [n_inactive, n_active],
            "histories_per_s": n / T, "seconds": T,
            "collisions_per_history": c["collisions"] / n,
            "k_col": [kc, sc], "k_site": [ks, ss],
            "sites_per_generation_last": int(out["n_sites"][-1])}


def bench_batch(args, torch, mcdc, W):
    """The batched workload on its own (one JSON line)."""
    r = batch_rate(torch, mcdc, W, args.steps, args.warmup)
    print(json.dumps({
        "metric": "histories/s, 256 batched problems (one persistent launch per census step, "
                  "graph-replayed)", "value": r["histories_per_s"], "unit": "histories/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_pass"],
        "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": r["workload"], "histories_per_pass": r["histories_per_pass"],
                   "autotuned_options": r["autotuned_options"],
                   "autotune_trials": r["autotune_trials"]},
        "pieces_per_history": r["pieces_per_history"]}), flush=True)


WW_MAP_DIMS = (30, 50, 30, 20)      # 2 cm cells x 10 s: network baked per cell centre


def fom_comparison(mcdc, W, analog_options, tile, target=0.01):
    """FOM = 1/(R^2 T) at `target` detector relative error on the duct
    problem: analog (the options of the main duct step) vs learned weight
    windows (importance from 20 x 1e6 analog histories, network trained on
    the GPU, baked onto a 2 cm x 10 s window map; schedule picked by the
    autotuner between the event and hybrid schedules, which spread long split
    chains over the grid; the analog hot tile where the schedule takes one).
    Each side: a pilot run sets N for the target error, then N histories are
    timed after a warm-up run.  The importance runs and the training, timed
    after a warm-up pass of that pipeline, are the setup that
    fom_with_training_amortised adds to the learned side's time; the map bake
    (part of that side's problem set-up) and the tuning are not added."""
    from paper_2409_04668_amd import learned_ww as L
    p = W.config2()
    # the setup is timed as the runs are, after a warm-up: a small pipeline
    # pass first loads the kernels it uses (reported beside the timed setup)
    t0 = time.perf_counter()
    L.build_ww(p, n_runs=1, n_per_run=100_000, steps=10, map_dims=WW_MAP_DIMS)
    t_warm = time.perf_counter() - t0
    t0 = time.perf_counter()
    ww, info = L.build_ww(p, n_runs=20, n_per_run=1_000_000, map_dims=WW_MAP_DIMS)
    t_build = time.perf_counter() - t0
    pw = W.config4(ww)
    # the autotuner picks the schedule for the weight-window problem from a
    # short pilot; resident histories for the event schedule then follow the
    # run length (up to 2^23)
    from paper_2409_04668_amd import autotune
    # the history schedule runs a history's whole split chain on one work-item
    # (1e6-1e7 histories/s with windows): not a candidate
    choice = autotune.tune_single(pw, pilot=4_000_000, waves=(16,), event_chunks=(1 << 22,),
                                  tile=tile, use_cache=False,
                                  schedules=(mcdc.SCHED_EVENT, mcdc.SCHED_HYBRID))
    wopt = dict(choice["options"])
    wopt["event_chunk"] = 1 << 25
    analog = L.fom_at_target(p, seed=31, target=target, pilot=20_000_000,
                             options=mcdc.make_options(**analog_options))
    learned = L.fom_at_target(pw, seed=41, target=target, pilot=4_000_000,
                              options=mcdc.make_options(**wopt))
    # the same network evaluated in the kernel at every window check (no map)
    pn = W.config4(dict(ww, map=None))
    net = L.fom_at_target(pn, seed=51, target=target, pilot=2_000_000,
                          options=mcdc.make_options(**wopt))

    def z(a, b):
        return abs(a["mean"] - b["mean"]) / ((a["mean"] * a["rel_err"]) ** 2 +
                                             (b["mean"] * b["rel_err"]) ** 2) ** 0.5
    return {"target_rel_err": target, "ratio": learned["fom"] / analog["fom"],
            "analog": dict(analog, schedule=SCHED_NAMES[analog_options["schedule"]],
                           options=analog_options),
            "learned_ww": dict(learned, window_map=list(WW_MAP_DIMS),
                               schedule=SCHED_NAMES[wopt["schedule"]], options=wopt,
                               autotune_trials=choice["trials"]),
            "learned_ww_network_per_check": dict(net, schedule=SCHED_NAMES[wopt["schedule"]],
                                                 ratio_to_analog=net["fom"] / analog["fom"]),
            "agreement_sigma": z(analog, learned),
            "agreement_sigma_network_per_check": z(analog, net),
            "training": dict(info, total_seconds=t_build, warmup_pass_seconds=t_warm,
                             flops_per_s=mlp_train_flops(info["n_points"], 5, 3000) /
                             info["train_seconds"]),
            "fom_with_training_amortised": 1.0 / (learned["rel_err"] ** 2 *
                                                  (learned["seconds"] + t_build))}


def mlp_train_flops(n_points, in_dim, steps, hidden=64):
    """Arithmetic of full-batch training: per point and step the forward pass
    (multiply and add of every weight: 2 (H in + H H + H)) and the backward
    pass (twice that: gradients with respect to weights and activations)."""
    fwd = 2 * (hidden * in_dim + hidden * hidden + hidden)
    return 3.0 * fwd * n_points * steps


def bench_fom(args, torch, mcdc, W):
    """FOM at 1% detector relative error, analog vs learned weight windows."""
    oargs, _, tile, _ = duct_options(args, mcdc, W.config2())
    f = fom_comparison(mcdc, W, oargs, tile)
    print(json.dumps({
        "metric": "FOM 1/(R^2 T) at 1% detector relative error, analog vs learned weight windows",
        "value": f["ratio"], "unit": "FOM ratio (learned / analog)", **f,
        "n_gpus": 1, "dtype": "f64", "data": "synthetic"}), flush=True)


if __name__ == "__main__":
    main()
