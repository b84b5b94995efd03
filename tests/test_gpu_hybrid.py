"""GPU parity of the hybrid schedule: a history-style lead stage (one
work-item follows each history, split daughters on its stack, for up to a
budget of flights or, under population control or census-step control, up to
the first census) followed by the event stages for what it banked.  Against the oracle on the same seeded inputs: identical
per-particle traces; per-history sums bit-identical where one particle
carries the history, to 1e-12 where split particles add into them in another
order; tally sums to 1e-10; integer counters exact."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_04668_amd import workloads as W

from gpu_util import assert_close_sums, assert_counters, assert_traces_equal, full_parity, run_pair
from test_gpu_parity import _col_box, _stepped_with_checkpoint, _void_pulse, _ww_box, ramp_mlp

pytestmark = pytest.mark.gpu


def _mcdc():
    from paper_2409_04668_amd import mcdc
    return mcdc


def _hy(chunk=0):
    mc = _mcdc()
    return mc.make_options(mc.SCHED_HYBRID, event_chunk=chunk)


def _split_pair(p, n, seed, chunk=0, trace_cap=400000):
    gp, orc, tg, to, hg, ho = run_pair(p, n, seed, trace_cap=trace_cap, options=_hy(chunk))
    assert_traces_equal(tg[0], to[0])
    np.testing.assert_allclose(hg[0], ho[0], rtol=1e-12, atol=1e-300)
    s, s2 = gp.raw()
    assert_close_sums(s, orc.tally_sum, what="tally_sum")
    assert_close_sums(s2, orc.tally_sumsq, what="tally_sumsq")
    if p.get("collision_tally"):
        c, _ = gp.raw_collision()
        assert_close_sums(c, orc.col_sum, what="col_sum")
    assert_counters(gp.counters(), orc)
    return gp, orc


def test_hybrid_slab_parity():
    full_parity(W.config1(), 3000, seed=171, trace_cap=60000, options=_hy())


def test_hybrid_duct_census_ragged_chunks_with_collision_tally():
    p = W.config2(n_census=5)
    p["mesh"]["n"] = np.array([12, 20, 12, 10], np.int32)
    p["collision_tally"] = True
    # chunks of 1000 histories: several chunks per batch, a ragged last chunk
    full_parity(p, 4321, seed=172, trace_cap=300000, options=_hy(1000))


def test_hybrid_multigroup_implicit_parity():
    p = W.config3()
    p["implicit_capture"] = True
    p["mesh"]["n"] = np.array([6, 10, 6, 5], np.int32)
    full_parity(p, 300, seed=173, trace_cap=600000, options=_hy())


def test_hybrid_two_materials_collision_tally():
    full_parity(_col_box(), 3000, seed=174, trace_cap=300000, options=_hy())


def test_hybrid_ragged_and_empty_runs():
    p = W.config1()
    for n in (0, 1, 7):
        full_parity(p, n, seed=175, trace_cap=1000, options=_hy())
    full_parity(p, 333, seed=176, trace_cap=20000, runs=3, options=_hy(100))


def test_hybrid_weight_windows_network():
    p = _ww_box()
    p["ww"] = dict(params=ramp_mlp(2.0, noise_seed=3), hidden=64, logk=0.0, ratio=5.0, n_max=10)
    gp, orc = _split_pair(p, 1500, 177)
    c = orc.counters
    assert c["split"] > 100 and c["rr_kill"] > 20


@pytest.mark.parametrize("stack_cap", [64, 2])
def test_hybrid_long_histories_hand_over_to_the_banks(stack_cap):
    """Scattering ratio 0.99 (about 100 flights per history) and a flat window
    w_T = 1/4 that splits every source particle into four at its first
    collision: the lead stage hands each history's particle and its stacked
    daughters to the banks after its flight budget; with a stack of two the
    third daughter goes straight to the bank.  Same trajectories as the
    oracle."""
    p = W.infinite_medium(1.0, [[0.99]], [1.0], half=5.0, t_end=150.0, nt=5)
    p["ww"] = dict(params=ramp_mlp(0.0), hidden=64, logk=float(np.log(0.25)), ratio=5.0, n_max=10)
    p["stack_cap"] = 64
    orc = O.OracleRun(p)
    to, ho = orc.run(200, 184, trace_cap=1_500_000, per_history=True)
    gp = _mcdc().Problem(dict(p, stack_cap=stack_cap), _hy())
    gp.set_trace(1_500_000)
    gp.set_history_scores(200)
    gp.run(200, 184)
    assert_traces_equal(gp.trace(), to)
    np.testing.assert_allclose(gp.history_scores(), ho, rtol=1e-12, atol=1e-300)
    s, _ = gp.raw()
    assert_close_sums(s, orc.tally_sum, what="tally_sum")
    assert_counters(gp.counters(), orc)
    c = orc.counters
    assert c["split"] % 3 == 0 and c["split"] > 500 and c["flight"] > 200 * 64
    # the banks were used: what the lead stage handed over took more than one
    # re-lead iteration (the first host check comes after one)
    assert gp.counters()["event_iterations"] > 1


def test_hybrid_event_cap_reached_in_the_re_lead_stage():
    """Histories of about 100 flights with a cap of 40: the lead stage hands
    each over after 32 flights and the re-lead stage, counting on from the
    history's stored count, reports the cap."""
    mc = _mcdc()
    p = W.infinite_medium(1.0, [[0.99]], [1.0], half=5.0, t_end=150.0, nt=5)
    p["ww"] = dict(params=ramp_mlp(0.0), hidden=64, logk=float(np.log(0.25)), ratio=5.0, n_max=10)
    p["max_events"] = 40
    gp = mc.Problem(p, _hy())
    gp.run(200, 184)
    with pytest.raises(mc.McdcError) as e:
        gp.tallies(mc.TALLY_MESH)
    assert e.value.status == mc.E_EVENT_CAP
    gp.close()
    p["max_events"] = 100000                        # the same run without the cap is clean
    gq = mc.Problem(p, _hy())
    gq.run(200, 184)
    gq.tallies(mc.TALLY_MESH)
    gq.close()


def test_hybrid_weight_window_map_duct_small_chunks():
    p = W.config2(n_census=3)
    p["mesh"]["n"] = np.array([6, 10, 6, 4], np.int32)
    p["ww"] = dict(params=ramp_mlp(-1.5, noise_seed=5), hidden=64, logk=0.3, ratio=5.0, n_max=10,
                   map=(12, 20, 12, 10))
    p["collision_tally"] = True
    gp, orc = _split_pair(p, 900, 178, chunk=256)
    assert orc.counters["split"] > 10


@pytest.mark.parametrize("target", [2.0, 0.3])
def test_hybrid_population_control_void(target):
    gp, orc = _split_pair(_void_pulse(target), 1000, 179)
    c = orc.counters
    assert c["pc_copy"] > 0 if target > 1 else c["pc_kill"] > 0


def test_hybrid_population_control_duct_with_weight_window_map():
    p = W.config2(n_census=4)
    p["mesh"]["n"] = np.array([6, 10, 6, 4], np.int32)
    p["ww"] = dict(params=ramp_mlp(-1.5, noise_seed=5), hidden=64, logk=0.3, ratio=5.0, n_max=10,
                   map=(12, 20, 12, 10))
    p["population_control"] = dict(target=0.7)
    gp, orc = _split_pair(p, 1500, 180)
    assert orc.counters["pc_kill"] > 0 and orc.counters["split"] > 0


def test_hybrid_census_steps_checkpoint_resume():
    """Census-step control stops the lead stage at the first census; a run
    copied into a fresh handle mid-way finishes with the oracle's results."""
    p = W.config2(n_census=5)
    p["mesh"]["n"] = np.array([12, 20, 12, 10], np.int32)
    n, seed = 4000, 181
    gb, steps, _ = _stepped_with_checkpoint(p, n, seed, _hy(1 << 13))
    assert 3 <= steps <= 6
    orc = O.OracleRun(p)
    _, ho = orc.run(n, seed, per_history=True)
    assert np.array_equal(gb.history_scores(), ho)
    s, s2 = gb.raw()
    assert_close_sums(s, orc.tally_sum, what="tally_sum")
    assert_close_sums(s2, orc.tally_sumsq, what="tally_sumsq")
    assert_counters(gb.counters(), orc)
    gb.close()


def test_hybrid_agrees_with_history_schedule_at_scale():
    """2e6 duct histories: per-history results identical to the history
    schedule's, bit for bit (one particle per history, same summation order)."""
    mc = _mcdc()
    p = W.config2(n_census=4)
    n = 2_000_000
    out = []
    for opt in (mc.make_options(mc.SCHED_HISTORY), _hy(1 << 20)):
        gp = mc.Problem(p, opt)
        gp.set_history_scores(n)
        gp.run(n, 182)
        out.append((gp.history_scores(), gp.raw(), gp.counters()))
        gp.close()
    (h1, s1, c1), (h2, s2, c2) = out
    assert np.array_equal(h1, h2)
    assert_close_sums(s1[0], s2[0], what="tally")
    assert_close_sums(s1[1], s2[1], what="tally_sumsq")
    for k in ("histories", "flights", "pieces", "collisions", "leaks", "census_stops", "time_ends"):
        assert c1[k] == c2[k], k


def test_hybrid_weight_window_map_matches_event_schedule_at_scale():
    """1e6 duct histories with a window map: the hybrid and the event schedule
    give the same per-history results (to 1e-12) and the same counts."""
    mc = _mcdc()
    p = W.config2()
    p["ww"] = dict(params=ramp_mlp(-1.5, noise_seed=5), hidden=64, logk=0.3, ratio=5.0, n_max=10,
                   map=(30, 50, 30, 20))
    n = 1_000_000
    out = []
    for opt in (mc.make_options(mc.SCHED_EVENT, event_chunk=1 << 20), _hy(1 << 18)):
        gp = mc.Problem(p, opt)
        gp.set_history_scores(n)
        gp.run(n, 183)
        out.append((gp.history_scores(), gp.raw(), gp.counters()))
        gp.close()
    (h1, s1, c1), (h2, s2, c2) = out
    np.testing.assert_allclose(h2, h1, rtol=1e-12, atol=1e-300)
    assert_close_sums(s1[0], s2[0], what="tally")
    for k in ("histories", "flights", "pieces", "collisions", "splits", "rr_kills", "particles",
              "leaks", "time_ends"):
        assert c1[k] == c2[k], k
    assert c1["splits"] > 1000


# ---------------------------------------------------------------------------
# LDS hot tile in the lead and re-lead stages (hybrid) and in the flight stage
# (event): one batch per workgroup tile
# ---------------------------------------------------------------------------

def _hy_tile(tile, chunk=0, sched="hybrid"):
    mc = _mcdc()
    return mc.make_options(mc.SCHED_HYBRID if sched == "hybrid" else mc.SCHED_EVENT,
                           event_chunk=chunk, tile=tile)


@pytest.mark.parametrize("sched", ["hybrid", "event"])
def test_hot_tile_duct_batches_straddle_workgroups(sched):
    """3000 histories in 20 batches of 150 over workgroup ranges of other
    sizes: a workgroup's range crosses batch boundaries, and the batch slices
    (sums of squares per batch) still match the oracle."""
    p = W.config2(n_census=3)
    tile = ([2, 3, 1, 0, 0], [10, 12, 9, 6, 1])        # x, y, z, t, g
    full_parity(p, 3000, seed=185, trace_cap=200000, options=_hy_tile(tile, sched=sched))


@pytest.mark.parametrize("sched", ["hybrid", "event"])
def test_hot_tile_multigroup_partial_groups_ragged_chunks(sched):
    p = W.config3()
    tile = ([0, 0, 0, 0, 3], [12, 12, 10, 2, 4])       # groups 3..6 only
    full_parity(p, 400, seed=186, trace_cap=300000, options=_hy_tile(tile, chunk=150, sched=sched))


@pytest.mark.parametrize("sched", ["hybrid", "event"])
def test_hot_tile_weight_window_map(sched):
    p = W.config2(n_census=3)
    p["ww"] = dict(params=ramp_mlp(-1.5, noise_seed=5), hidden=64, logk=0.3, ratio=5.0, n_max=10,
                   map=(12, 20, 12, 10))
    p["collision_tally"] = True
    tile = ([0, 0, 0, 0, 0], [16, 20, 10, 4, 1])
    gp, orc, tg, to, hg, ho = run_pair(p, 900, 187, trace_cap=400000, options=_hy_tile(tile, sched=sched))
    assert_traces_equal(tg[0], to[0])
    np.testing.assert_allclose(hg[0], ho[0], rtol=1e-12, atol=1e-300)
    s, s2 = gp.raw()
    assert_close_sums(s, orc.tally_sum, what="tally_sum")
    assert_close_sums(s2, orc.tally_sumsq, what="tally_sumsq")
    assert_counters(gp.counters(), orc)
    assert orc.counters["split"] > 10


@pytest.mark.parametrize("sched", ["hybrid", "event"])
def test_hot_tile_with_population_control(sched):
    """Population control at four census steps of the duct with the LDS hot
    tile: census stops from the tiled flight stage (event) or the lead and
    re-lead stages (hybrid), the control between steps; trajectories as the
    oracle's, tallies and their batch slices to 1e-10."""
    p = W.config2(n_census=4)
    p["mesh"]["n"] = np.array([12, 20, 12, 8], np.int32)
    p["population_control"] = dict(target=1.3)
    p["n_batches"] = 2
    tile = ([2, 3, 1, 0, 0], [8, 10, 8, 4, 1])
    gp, orc, tg, to, hg, ho = run_pair(p, 2000, 189, trace_cap=600000,
                                       options=_hy_tile(tile, chunk=1 << 11, sched=sched))
    assert_traces_equal(tg[0], to[0])
    np.testing.assert_allclose(hg[0], ho[0], rtol=1e-12, atol=1e-300)
    s, s2 = gp.raw()
    assert_close_sums(s, orc.tally_sum, what="tally_sum")
    assert_close_sums(s2, orc.tally_sumsq, what="tally_sumsq")
    assert_counters(gp.counters(), orc)
    assert orc.counters["pc_copy"] + orc.counters["pc_kill"] > 100


def test_planned_tile_at_scale_matches_history_schedule():
    """The autotuner's tile for the full duct problem, 5e6 histories: the
    hybrid and event schedules with the tile give the history schedule's
    per-history results bit for bit and its tallies to reordering."""
    mc = _mcdc()
    from paper_2409_04668_amd import autotune
    p = W.config2()
    tile, frac = autotune.plan_hot_tile(p, pilot=1_000_000)
    assert tile is not None and frac > 0.5
    n = 5_000_000
    res = []
    for opt in (mc.make_options(mc.SCHED_HISTORY, tile=tile), _hy_tile(tile, chunk=1 << 22),
                _hy_tile(tile, chunk=1 << 22, sched="event")):
        gp = mc.Problem(p, opt)
        gp.set_history_scores(n)
        gp.run(n, 188)
        res.append((gp.history_scores(), gp.raw(), gp.counters()))
        gp.close()
    for other in res[1:]:
        assert np.array_equal(res[0][0], other[0])
        assert_close_sums(res[0][1][0], other[1][0], what="tally")
        assert_close_sums(res[0][1][1], other[1][1], what="tally_sumsq")
        assert res[0][2]["pieces"] == other[2]["pieces"]


def test_full_size_duct_hybrid_tile_sampled_histories():
    """The duct problem at full size (1e8 histories) in the launch
    configuration the benchmark's autotuner picks on this GPU: the hybrid
    schedule, 2^25 resident histories, the LDS hot tile from the analog pilot.
    Sampled histories recomputed one by one by the oracle match bit for bit;
    all track length is scored and weight balances."""
    from paper_2409_04668_amd import autotune
    mc = _mcdc()
    n = 100_000_000
    p = W.config2()
    tile, _ = autotune.plan_hot_tile(p, pilot=1_000_000)
    gp = mc.Problem(p, _hy_tile(tile, chunk=1 << 25))
    gp.set_history_scores(n)
    gp.run(n, seed=2028)
    hs = gp.history_scores()
    rng = np.random.default_rng(1)
    # histories at chunk and workgroup-range edges, random ones, detector hits
    ids = np.unique(np.concatenate([[0, 1, (1 << 25) - 1, 1 << 25, n - 1], rng.integers(0, n, 40),
                                    np.nonzero(hs[:, 0] > 0)[0][:20]]))
    q = dict(p)
    q["n_batches"] = 1
    for i in ids:
        r = O.OracleRun(q)
        _, ho = r.run(1, 2028, per_history=True, first_id=int(i))
        assert np.array_equal(ho[0], hs[i]), (i, ho[0], hs[i])
    c = gp.counters()
    s, _ = gp.raw()
    gp.close()
    assert c["histories"] == n and c["particles"] == n
    assert abs(s.sum() - c["path"]) <= 1e-9 * c["path"]
    assert c["w_source"] == c["w_leak"] + c["w_absorb"] + c["w_time_end"]
    assert c["leaks"] + c["absorptions"] + c["time_ends"] == n


def test_full_size_multigroup_duct_hybrid_sampled_histories():
    """The 7-group duct at full size (1e8 histories, 60x100x60 x 20 t x 7 groups
    = 5.04e7 bins, per-batch slices), hybrid schedule with the tile the
    autotuner plans for it: sampled histories recomputed one by one by the
    oracle match bit for bit; all track length is scored and weight balances."""
    from paper_2409_04668_amd import autotune
    mc = _mcdc()
    n = 100_000_000
    p = W.config3()
    tile, frac = autotune.plan_hot_tile(p, pilot=1_000_000)
    assert tile is not None and frac > 0.0
    gp = mc.Problem(p, _hy_tile(tile, chunk=1 << 25))
    gp.set_history_scores(n)
    gp.run(n, seed=2029)
    hs = gp.history_scores()
    c = gp.counters()
    s, _ = gp.raw()
    gp.close()
    rng = np.random.default_rng(2)
    ids = np.unique(np.concatenate([[0, (1 << 25) - 1, 1 << 25, n - 1], rng.integers(0, n, 24),
                                    np.nonzero(hs[:, 0] > 0)[0][:8]]))
    q = dict(p)
    q["n_batches"] = 1
    for i in ids:
        r = O.OracleRun(q)
        _, ho = r.run(1, 2029, per_history=True, first_id=int(i))
        assert np.array_equal(ho[0], hs[i]), (i, ho[0], hs[i])
    assert c["histories"] == n and c["particles"] == n
    assert abs(s.sum() - c["path"]) <= 1e-9 * c["path"]
    assert c["w_source"] == c["w_leak"] + c["w_absorb"] + c["w_time_end"]


@pytest.mark.parametrize("config,n", [("duct", 2_000_000), ("duct7", 200_000)])
def test_headline_launch_configuration_full_mesh_tally(config, n):
    """The benchmark's launch configuration (hybrid schedule, 2^25 resident
    histories, the hot tile the autotuner plans from an analog pilot) against
    the oracle on the whole mesh: every one of the 7.2e6 bins (5.04e7 with
    seven groups) of tally_sum and tally_sumsq to 1e-10 with the same zero
    pattern, every history's (detector score, path) bit for bit, counters
    exact."""
    from paper_2409_04668_amd import autotune
    mc = _mcdc()
    p = W.config2() if config == "duct" else W.config3()
    tile, _ = autotune.plan_hot_tile(p, pilot=1_000_000)
    assert tile is not None
    gp = mc.Problem(p, _hy_tile(tile, chunk=1 << 25))
    orc = O.OracleRun(p)
    gp.set_history_scores(n)
    gp.run(n, 2031)
    _, ho = orc.run(n, 2031, per_history=True)
    assert np.array_equal(gp.history_scores(), ho)
    s, s2 = gp.raw()
    assert_close_sums(s, orc.tally_sum, what="tally_sum")
    assert_close_sums(s2, orc.tally_sumsq, what="tally_sumsq")
    assert_counters(gp.counters(), orc)
    gp.close()


@pytest.mark.parametrize("sched", ["history", "hybrid", "event"])
def test_full_size_slab_every_history(sched):
    """The slab problem at its full size (1e5 histories, 100 x-bins x 20
    t-bins): every history's (detector score, path) bit for bit, tallies and
    batch sums of squares to 1e-10, counters exact, under each schedule."""
    mc = _mcdc()
    opt = mc.make_options({"history": mc.SCHED_HISTORY, "hybrid": mc.SCHED_HYBRID,
                           "event": mc.SCHED_EVENT}[sched])
    full_parity(W.config1(), 100_000, seed=2030, options=opt)
