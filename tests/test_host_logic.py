"""Host-side logic that needs no GPU: the autotuner's hot-tile planner and the
workload generators."""
import numpy as np

from paper_2409_04668_amd import workloads as W


def test_grow_tile_finds_planted_box():
    from paper_2409_04668_amd.autotune import grow_tile
    rng = np.random.default_rng(0)
    D = 0.001 * rng.random((2, 20, 30, 40, 30))
    D[1, 3:7, 5:15, 10:22, 4:16] += 1.0 + rng.random((4, 10, 12, 12))
    (lo, n), frac = grow_tile(D, 4 * 10 * 12 * 12)
    assert list(lo) == [4, 10, 5, 3, 1] and list(n) == [12, 12, 10, 4, 1]
    assert frac > 0.9
    (lo2, n2), _ = grow_tile(D, 100)
    assert int(np.prod(n2)) <= 100


def test_config_shapes():
    assert W.n_bins(W.config1()) == 2000
    assert W.n_bins(W.config2()) == 60 * 100 * 60 * 20
    assert W.n_bins(W.config3()) == 60 * 100 * 60 * 20 * 7
    p3 = W.config3()
    rows = p3["sigma_s"].sum(axis=2)
    assert np.all(rows <= p3["sigma_t"] * 0.9 + 1e-15) and np.all(rows >= p3["sigma_t"] * 0.3 - 1e-15)
    assert np.all(np.triu(p3["sigma_s"][0], 1) == 0)          # downscatter only
    probs, nh = W.config5()
    assert len(probs) == 256 and nh.min() >= 10_000 and nh.max() <= 1_000_000
    for p in probs[:20]:
        assert 1 <= p["sigma_t"].shape[1] <= 7 and p["mesh"]["n"][3] == len(p["census"]) == 10
        assert 0 <= len(p["box_mat"]) <= 7


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: any other --gpus exits with status 2 and a
    message, before touching a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_committed_profiles_match_the_kernel_sources():
    """The PMC and SQ summaries the benchmark reads carry the hash of the
    kernel sources they were taken with and the histories per launch; they
    match the current sources, and a changed launch size is refused."""
    import bench
    t = bench.measured_traffic("k_ev_lead", 1e8 / 3)
    assert t is not None and 1e9 < t < 2e10
    assert bench.measured_traffic("k_ev_lead", 1e8 / 6) is None
    assert bench.measured_traffic("k_history", 5e6) is not None
    v = bench.measured_valu("k_ev_lead")
    assert v is not None and 0 < v["lane_throughput_fraction"] <= v["simd_valu_busy_fraction"] <= 1


def test_tuner_trial_options_carry_the_tile(monkeypatch):
    """tune_single's trial list on the host (timings stubbed): every trial
    takes the tile (history kernel, lead and re-lead stages, event flight
    stage), and population control skips the history schedule and chunks
    below a batch."""
    from paper_2409_04668_amd import autotune, mcdc
    monkeypatch.setattr(autotune, "_time_single", lambda prob, opt, n, seed: float(opt.schedule))
    monkeypatch.setattr(autotune, "_device_name", lambda: "test")
    tile = ([1, 2, 3, 0, 0], [4, 5, 6, 2, 1])
    res = autotune.tune_single(W.config2(), pilot=1000, waves=(8, 16), event_chunks=(1 << 10,),
                               tile=tile, use_cache=False)
    opts = [t["options"] for t in res["trials"]]
    assert [o["schedule"] for o in opts] == [mcdc.SCHED_HISTORY] * 2 + [mcdc.SCHED_EVENT,
                                                                       mcdc.SCHED_HYBRID]
    for o in opts:
        assert "tile" in o
    assert res["options"]["schedule"] == mcdc.SCHED_HYBRID      # the stub's largest rate
    p = W.config2()
    p["population_control"] = dict(target=1.0)
    res = autotune.tune_single(p, pilot=100_000, event_chunks=(1 << 10, 1 << 16), use_cache=False)
    assert [t["options"]["event_chunk"] for t in res["trials"]] == [1 << 16, 1 << 16]


def test_keff_tuner_trial_options(monkeypatch):
    """tune_keff's trial list on the host (timings stubbed): the history
    schedule at each occupancy, then the hot tile; the pick is the fastest.
    No tile is planned when the mesh fits the whole-mesh LDS tally (and then
    no GPU run is made)."""
    from paper_2409_04668_amd import autotune, mcdc
    monkeypatch.setattr(autotune, "_time_keff",
                        lambda prob, opt, m, gens, seed: 100.0 if opt.tile_n[0] else float(opt.waves_per_cu))
    monkeypatch.setattr(autotune, "_device_name", lambda: "test")
    tile = ([1, 2, 2, 0, 1], [28, 26, 26, 1, 1])
    res = autotune.tune_keff(W.keff_core(nx=30), 1000, waves=(4, 8, 16), tile=tile, use_cache=False)
    opts = [t["options"] for t in res["trials"]]
    assert [o.get("waves_per_cu") for o in opts] == [4, 8, 16, None]
    assert all(o["schedule"] == mcdc.SCHED_HISTORY for o in opts)
    assert opts[-1]["tile"] == [list(tile[0]), list(tile[1])]
    assert res["options"] == opts[-1] and res["histories_per_s"] == 100.0
    res = autotune.tune_keff(W.keff_core(nx=30), 1000, waves=(4, 8), use_cache=False)
    assert res["options"]["waves_per_cu"] == 8 and len(res["trials"]) == 2
    assert autotune.plan_keff_tile(W.keff_core(nx=12)) == (None, 0.0)
