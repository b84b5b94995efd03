"""GPU tests of the autotuner: the schedule it picks runs the problem to the
same per-history results as any other schedule, population control is only
tried in the event and hybrid schedules, the batched tuner returns a working
shape, and the k-eigenvalue tuner's pick runs the same generations."""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2409_04668_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ramp(slope):
    prm = np.zeros(M.n_params(5, 64), np.float32)
    prm[0] = 1.0                            # W1[0][0]
    prm[64 * 5] = 1.0                       # b1[0]
    prm[64 * 5 + 64] = 1.0                  # W2[0][0]
    prm[64 * 5 + 64 + 64 * 64 + 64] = slope  # W3[0]
    prm[-1] = -slope                        # b3
    return prm


def test_tuned_schedule_gives_the_same_histories():
    from paper_2409_04668_amd import autotune, mcdc
    p = W.config2()
    p["mesh"]["n"] = np.array([6, 10, 6, 4], np.int32)
    p["ww"] = dict(params=_ramp(-1.5), hidden=64, logk=0.3, ratio=5.0, n_max=10,
                   map=(12, 20, 12, 10))
    p["stack_cap"] = 256
    res = autotune.tune_single(p, pilot=200_000, waves=(8, 16), event_chunks=(1 << 18,),
                               use_cache=False)
    assert len(res["trials"]) == 4 and res["histories_per_s"] > 0
    n = 20_000
    out = []
    for opt in (mcdc.make_options(**res["options"]), mcdc.make_options(mcdc.SCHED_HISTORY)):
        gp = mcdc.Problem(p, opt)
        gp.set_history_scores(n)
        gp.run(n, 5)
        out.append((gp.history_scores(), gp.counters()))
        gp.close()
    np.testing.assert_allclose(out[0][0], out[1][0], rtol=1e-12, atol=1e-300)
    for k in ("flights", "pieces", "splits", "rr_kills", "particles"):
        assert out[0][1][k] == out[1][1][k], k


def test_population_control_is_tuned_in_the_banked_schedules_only():
    from paper_2409_04668_amd import autotune, mcdc
    p = W.infinite_medium(1.0, [[0.8]], [1.0], half=20.0, t_end=8.0, nt=8)
    p["census"] = np.linspace(1.0, 8.0, 8)
    p["population_control"] = dict(target=1.0)
    res = autotune.tune_single(p, pilot=100_000, event_chunks=(1 << 12, 1 << 16),
                               use_cache=False)
    # batches of 5000 histories: the 4096 chunk cannot hold one
    assert [t["options"]["event_chunk"] for t in res["trials"]] == [1 << 16] * 2
    assert res["options"]["schedule"] in (mcdc.SCHED_EVENT, mcdc.SCHED_HYBRID)


def test_batch_tuner_returns_a_working_shape():
    from paper_2409_04668_amd import autotune, mcdc
    probs, n_hist = W.config5()
    probs, n_hist = probs[:12], np.minimum(n_hist[:12], 20_000)
    res = autotune.tune_batch(probs, n_hist, chunks=(512, 4096), waves=(8,), use_cache=False)
    assert len(res["trials"]) == 2 and res["histories_per_s"] > 0
    bp = mcdc.BatchProblem(probs, n_hist, mcdc.make_options(**res["options"]))
    bp.run(3)
    for i in range(len(probs)):
        assert bp.counters(i)["histories"] == n_hist[i]
    bp.close()


def test_tuner_gives_the_tile_to_every_trial():
    from paper_2409_04668_amd import autotune, mcdc
    p = W.config2(n_census=3)
    tile = ([2, 3, 1, 0, 0], [10, 12, 9, 6, 1])
    res = autotune.tune_single(p, pilot=200_000, waves=(16,), event_chunks=(1 << 18,), tile=tile,
                               use_cache=False)
    scheds = [t["options"]["schedule"] for t in res["trials"]]
    assert scheds == [mcdc.SCHED_HISTORY, mcdc.SCHED_EVENT, mcdc.SCHED_HYBRID]
    for t in res["trials"]:
        assert t["options"]["tile"] == [list(tile[0]), list(tile[1])]
    gp = mcdc.Problem(p, mcdc.make_options(**res["options"]))
    gp.run(10_000, 3)
    assert gp.counters()["histories"] == 10_000
    gp.close()


def test_keff_tuner_pick_runs_the_same_generations():
    """The k-eigenvalue tuner (occupancy for the generation size, a hot tile
    planned from a k-eigenvalue pilot) picks options that run the same
    generations as the defaults: the same site counts and site estimates bit
    for bit (trajectories do not depend on the grid or the tile), the
    collision estimate to float-atomic summation order."""
    from paper_2409_04668_amd import autotune, mcdc
    p = W.keff_core(nx=30)
    tile, frac = autotune.plan_keff_tile(p, m=20_000, generations=3)
    assert tile is not None and 0.0 < frac <= 1.0
    res = autotune.tune_keff(p, 20_000, waves=(4, 16), tile=tile, use_cache=False)
    assert len(res["trials"]) == 3 and res["histories_per_s"] > 0
    outs = []
    for opt in (mcdc.make_options(**res["options"]), mcdc.make_options(mcdc.SCHED_HISTORY)):
        gp = mcdc.Problem(p, opt)
        outs.append(gp.run_keff(20_000, 2, 3, seed=8))
        gp.close()
    np.testing.assert_array_equal(outs[0]["n_sites"], outs[1]["n_sites"])
    np.testing.assert_array_equal(outs[0]["k_site"], outs[1]["k_site"])
    np.testing.assert_allclose(outs[0]["k_col"], outs[1]["k_col"], rtol=1e-12)
