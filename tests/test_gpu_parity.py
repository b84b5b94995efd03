"""GPU parity: the HIP history kernel against the CPU oracle on the same seeded
inputs.  Per-history traces and per-history (detector score, path) must be
bit-identical; tally sums agree to 1e-10 relative (only the order of FP64
additions differs); integer counters are exact."""
import numpy as np
import pytest

from oracle import mlp as M
from oracle import oracle as O
from paper_2409_04668_amd import workloads as W

from gpu_util import assert_close_sums, full_parity, run_pair

pytestmark = pytest.mark.gpu


def _mcdc():
    from paper_2409_04668_amd import mcdc
    return mcdc


@pytest.mark.parametrize("lds", [1, 0])
def test_slab_history_parity(lds):
    mc = _mcdc()
    full_parity(W.config1(), 3000, seed=101, trace_cap=60000,
                options=mc.make_options(mc.SCHED_HISTORY, lds_tally=lds))


def test_slab_implicit_capture_parity():
    p = W.config1()
    p["implicit_capture"] = True
    full_parity(p, 2000, seed=102, trace_cap=200000)


def test_duct_parity_with_census_steps():
    p = W.config2(n_census=4)
    p["mesh"]["n"] = np.array([12, 20, 12, 8], np.int32)     # several tiles, ragged vs census
    full_parity(p, 3000, seed=103, trace_cap=200000)


def test_duct_full_mesh_parity():
    full_parity(W.config2(), 2000, seed=104, trace_cap=100000)


def test_multigroup_parity():
    p = W.config3()
    full_parity(p, 400, seed=105, trace_cap=200000)


def test_multigroup_implicit_parity():
    p = W.config3()
    p["implicit_capture"] = True
    p["mesh"]["n"] = np.array([6, 10, 6, 5], np.int32)
    full_parity(p, 200, seed=106, trace_cap=400000)


def test_reflective_infinite_medium_parity():
    p = W.infinite_medium([0.5, 0.8, 1.0], [[0.3, 0, 0], [0.2, 0.4, 0], [0.1, 0.3, 0.5]],
                          [1.0, 3.0, 10.0], half=2.0, t_end=3.0, nt=6)
    p["mesh"]["n"] = np.array([4, 4, 4, 6], np.int32)
    full_parity(p, 500, seed=107, trace_cap=400000)


def _ww_box():
    p = W._base(1)
    p["outer_lo"] = np.zeros(3)
    p["outer_hi"] = np.full(3, 20.0)
    p["sigma_t"] = np.array([[0.5]])
    p["sigma_s"] = np.array([[[0.4]]])
    p["source"] = dict(kind="point", lo=np.full(3, 10.0), hi=np.full(3, 10.0), t0=0.0, t1=0.0,
                       isotropic=True, dir=np.array([1.0, 0.0, 0.0]), group=0)
    p["mesh"] = dict(lo=np.array([0.0, 0.0, 0.0, 0.0]), hi=np.array([20.0, 20.0, 20.0, 40.0]),
                     n=np.array([10, 5, 5, 4], np.int32), per_group=False)
    p["census"] = np.array([40.0])
    p["detector"] = dict(lo=np.array([16.0, 0.0, 0.0]), hi=np.array([20.0, 20.0, 20.0]))
    return p


def ramp_mlp(slope, noise_seed=None):
    """y = slope * xhat_x (one ReLU path), optionally plus a small random net."""
    prm = np.zeros(M.n_params(5, 64), np.float32)
    o = 0
    prm[o] = 1.0                            # W1[0][0]
    o += 64 * 5
    prm[o] = 1.0                            # b1[0]
    o += 64
    prm[o] = 1.0                            # W2[0][0]
    o += 64 * 64 + 64
    prm[o] = slope                          # W3[0]
    o += 64
    prm[o] = -slope                         # b3
    if noise_seed is not None:
        noise = M.init_params(5, 64, seed=noise_seed) * np.float32(0.02)
        noise[0] = noise[64 * 5] = noise[64 * 5 + 64] = 0.0
        prm = prm + noise
    return prm


def test_weight_window_parity_ramp_mlp():
    p = _ww_box()
    p["ww"] = dict(params=ramp_mlp(2.0, noise_seed=3), hidden=64, logk=0.0, ratio=5.0, n_max=10,
                   ymin=-1.5, ymax=1.5)        # the clamp binds near both x faces
    p["stack_cap"] = 256
    gp, orc = full_parity(p, 1500, seed=108, trace_cap=400000)
    c = orc.counters
    assert c["split"] > 100 and c["rr_kill"] > 20


def test_weight_window_parity_duct():
    p = W.config2()
    p["mesh"]["n"] = np.array([6, 10, 6, 4], np.int32)
    p["ww"] = dict(params=ramp_mlp(-1.5, noise_seed=5), hidden=64, logk=0.3, ratio=5.0, n_max=10)
    p["stack_cap"] = 256
    gp, orc = full_parity(p, 800, seed=109, trace_cap=400000)
    assert orc.counters["split"] > 10


def test_ww_map_bake_bit_exact():
    """The device bake of the window map equals the oracle's map bit for bit."""
    mc = _mcdc()
    p = _ww_box()
    p["ww"] = dict(params=M.init_params(5, 64, seed=21), hidden=64, logk=0.2, ratio=5.0,
                   n_max=10, ymin=-0.4, ymax=0.6, map=(7, 5, 3, 4))
    p["stack_cap"] = 256
    gp = mc.Problem(p)
    got = gp.ww_map()
    want = O.ww_map(p).reshape(-1)
    assert got.shape == want.shape and np.array_equal(got, want)
    gp.close()


def test_ww_map_parity_history():
    p = _ww_box()
    p["ww"] = dict(params=ramp_mlp(2.0, noise_seed=3), hidden=64, logk=0.0, ratio=5.0, n_max=10,
                   ymin=-1.5, ymax=1.5, map=(10, 4, 4, 8))
    p["stack_cap"] = 256
    gp, orc = full_parity(p, 1500, seed=110, trace_cap=400000)
    c = orc.counters
    assert c["split"] > 100 and c["rr_kill"] > 20


def test_ww_map_parity_duct_event():
    """Duct with a baked map under the event schedule: identical trajectories."""
    from gpu_util import assert_counters, assert_traces_equal, run_pair
    p = W.config2()
    p["mesh"]["n"] = np.array([6, 10, 6, 4], np.int32)
    p["ww"] = dict(params=ramp_mlp(-1.5, noise_seed=5), hidden=64, logk=0.3, ratio=5.0, n_max=10,
                   map=(12, 20, 12, 10))
    p["stack_cap"] = 256
    gp, orc, tg, to, hg, ho = run_pair(p, 800, 111, trace_cap=400000, options=_ev())
    assert_traces_equal(tg[0], to[0])
    np.testing.assert_allclose(hg[0], ho[0], rtol=1e-12, atol=0)
    s, s2 = gp.raw()
    assert_close_sums(s, orc.tally_sum, what="tally_sum")
    assert_counters(gp.counters(), orc)
    assert orc.counters["split"] > 10


# ---------------------------------------------------------------------------
# event-based schedule: same per-particle trajectories, other execution order
# ---------------------------------------------------------------------------

def _ev(chunk=0):
    mc = _mcdc()
    return mc.make_options(mc.SCHED_EVENT, event_chunk=chunk)


def test_event_schedule_slab_parity():
    full_parity(W.config1(), 3000, seed=121, trace_cap=60000, options=_ev())


def test_event_schedule_duct_census_parity_small_chunks():
    p = W.config2(n_census=5)
    p["mesh"]["n"] = np.array([12, 20, 12, 10], np.int32)
    # chunks of 1000 histories: several chunks per batch and a ragged last chunk
    full_parity(p, 4321, seed=122, trace_cap=300000, options=_ev(1000))


def test_event_schedule_multigroup_implicit_parity():
    p = W.config3()
    p["implicit_capture"] = True
    p["mesh"]["n"] = np.array([6, 10, 6, 5], np.int32)
    full_parity(p, 300, seed=123, trace_cap=600000, options=_ev())


def test_event_schedule_weight_windows():
    """With splitting, a history's particles run in another order, so the
    per-history sums may round differently; trajectories stay identical."""
    from gpu_util import assert_counters, assert_traces_equal, run_pair
    p = _ww_box()
    p["ww"] = dict(params=ramp_mlp(2.0, noise_seed=3), hidden=64, logk=0.0, ratio=5.0, n_max=10)
    p["stack_cap"] = 256
    gp, orc, tg, to, hg, ho = run_pair(p, 1500, 124, trace_cap=400000, options=_ev())
    assert_traces_equal(tg[0], to[0])
    np.testing.assert_allclose(hg[0], ho[0], rtol=1e-12, atol=0)
    s, s2 = gp.raw()
    assert_close_sums(s, orc.tally_sum, what="tally_sum")
    assert_close_sums(s2, orc.tally_sumsq, what="tally_sumsq")    # batch slices
    assert_counters(gp.counters(), orc)


def test_history_and_event_schedules_agree_at_scale():
    """2e6 duct histories: both schedules give identical per-history results."""
    mc = _mcdc()
    p = W.config2(n_census=4)
    n = 2_000_000
    out = []
    for opt in (mc.make_options(mc.SCHED_HISTORY), _ev(1 << 20)):
        gp = mc.Problem(p, opt)
        gp.set_history_scores(n)
        gp.run(n, 31)
        out.append((gp.history_scores(), gp.raw(), gp.counters()))
        gp.close()
    (h1, s1, c1), (h2, s2, c2) = out
    assert np.array_equal(h1, h2)
    assert_close_sums(s1[0], s2[0], what="tally")
    assert_close_sums(s1[1], s2[1], what="tally_sumsq")
    for k in ("histories", "flights", "pieces", "collisions", "leaks", "census_stops", "time_ends"):
        assert c1[k] == c2[k], k


def test_importance_estimate_parity():
    p = W.config2()
    p["mesh"]["n"] = np.array([6, 10, 6, 4], np.int32)
    p["importance"] = W.coarse_importance_grid()
    gp, orc = full_parity(p, 4000, seed=110)
    s, w = gp.importance()
    assert_close_sums(s, orc.imp_score, what="imp_score")
    assert_close_sums(w, orc.imp_weight, what="imp_weight")


def test_ragged_and_accumulating_runs():
    p = W.config1()
    # fewer histories than batches, then more runs continuing the history ids
    for n in (0, 1, 7):
        full_parity(p, n, seed=111, trace_cap=1000)
    full_parity(p, 333, seed=112, trace_cap=20000, runs=3)


def test_event_cap_reports_error():
    mc = _mcdc()
    p = W.infinite_medium(1.0, [[0.99]], [1.0], half=5.0, t_end=1e6, nt=1)
    p["max_events"] = 5
    gp = mc.Problem(p)
    gp.run(100, 1)
    with pytest.raises(mc.McdcError) as e:
        gp.tallies(mc.TALLY_DETECTOR)
    assert e.value.status == mc.E_EVENT_CAP
    with pytest.raises(O.OracleError):
        O.run(p, 100, 1)


def test_invalid_desc_rejected():
    mc = _mcdc()
    p = W.config1()
    p["census"] = np.array([5.0, 4.0])
    with pytest.raises(mc.McdcError) as e:
        mc.Problem(p)
    assert e.value.status == mc.E_INVALID


def test_full_size_duct_sampled_histories():
    """Config-2 at full size (1e8 histories, bench launch configuration: the
    history schedule with the LDS hot tile the autotuner places): sampled
    histories recomputed one by one by the oracle match bit for bit; all
    track length is scored (conservation) and weight balances."""
    from paper_2409_04668_amd import autotune
    mc = _mcdc()
    n = 100_000_000
    p = W.config2()
    tile, _ = autotune.plan_hot_tile(p, pilot=1_000_000)
    gp = mc.Problem(p, mc.make_options(mc.SCHED_HISTORY, tile=tile))
    gp.set_history_scores(n)
    gp.run(n, seed=2026)
    hs = gp.history_scores()
    rng = np.random.default_rng(0)
    ids = np.unique(np.concatenate([[0, 1, n - 1], rng.integers(0, n, 40),
                                    np.nonzero(hs[:, 0] > 0)[0][:20]]))
    q = dict(p)
    q["n_batches"] = 1
    for i in ids:
        r = O.OracleRun(q)
        _, ho = r.run(1, 2026, per_history=True, first_id=int(i))
        assert np.array_equal(ho[0], hs[i]), (i, ho[0], hs[i])
    c = gp.counters()
    s, _ = gp.raw()
    assert c["histories"] == n and c["particles"] == n
    assert abs(s.sum() - c["path"]) <= 1e-9 * c["path"]
    assert c["w_source"] == c["w_leak"] + c["w_absorb"] + c["w_time_end"]
    assert c["leaks"] + c["absorptions"] + c["time_ends"] == n


@pytest.fixture(scope="module")
def learned_duct_ww():
    from paper_2409_04668_amd import learned_ww as L
    p = W.config2()
    ww, _ = L.build_ww(p, n_runs=4, n_per_run=1_000_000, steps=600, map_dims=(30, 50, 30, 20))
    return W.config4(ww)


@pytest.mark.slow
@pytest.mark.parametrize("schedule", ["event", "hybrid"])
def test_full_size_learned_ww_sampled_histories(learned_duct_ww, schedule):
    """The learned weight-window configuration as the FOM comparison runs it
    (trained network baked onto the 2 cm x 10 s map) at 4e7 histories, under
    the event schedule (2^23 resident histories) and under the hybrid
    schedule the autotuner picks on this GPU (2^25 resident histories, the
    analog run's LDS hot tile): blocks of histories recomputed by the oracle
    agree per history (several particles add into a history's sums in
    another order: 1e-12); weight balances over the whole run."""
    from paper_2409_04668_amd import autotune
    mc = _mcdc()
    pw = learned_duct_ww
    n = 40_000_000
    if schedule == "event":
        opt = mc.make_options(mc.SCHED_EVENT, event_chunk=1 << 23)
    else:
        tile, _ = autotune.plan_hot_tile(W.config2(), pilot=1_000_000)
        opt = mc.make_options(mc.SCHED_HYBRID, event_chunk=1 << 25, tile=tile)
    gp = mc.Problem(pw, opt)
    gp.set_history_scores(n)
    gp.run(n, seed=2027)
    hs = gp.history_scores()
    c = gp.counters()
    gp.close()
    hit = int(np.nonzero(hs[:, 0] > 0)[0][0])
    q = dict(pw)
    q["n_batches"] = 1
    for first in (0, hit, (1 << 25) - 20, n - 40):
        r = O.OracleRun(q)
        _, ho = r.run(40, 2027, per_history=True, first_id=first)
        np.testing.assert_allclose(hs[first:first + 40], ho, rtol=1e-12, atol=1e-300)
    assert c["histories"] == n and c["splits"] > 0
    lhs = c["w_source"] + c["w_gain"] - c["w_loss"]
    rhs = c["w_leak"] + c["w_absorb"] + c["w_time_end"]
    assert abs(lhs - rhs) <= 1e-9 * c["w_source"]


# ---------------------------------------------------------------------------
# LDS hot tile: a sub-box of the mesh privatised per workgroup
# ---------------------------------------------------------------------------

def test_hot_tile_parity_duct():
    mc = _mcdc()
    p = W.config2(n_census=3)
    tile = ([2, 3, 1, 0, 0], [10, 12, 9, 6, 1])        # x, y, z, t, g
    full_parity(p, 3000, seed=131, trace_cap=200000,
                options=mc.make_options(mc.SCHED_HISTORY, tile=tile))


def test_hot_tile_parity_multigroup_partial_groups():
    mc = _mcdc()
    p = W.config3()
    tile = ([0, 0, 0, 0, 3], [12, 12, 10, 2, 4])       # groups 3..6 only
    full_parity(p, 400, seed=132, trace_cap=300000,
                options=mc.make_options(mc.SCHED_HISTORY, tile=tile))


def test_hot_tile_rejects_outside_mesh():
    mc = _mcdc()
    with pytest.raises(mc.McdcError) as e:
        mc.Problem(W.config2(), mc.make_options(tile=([55, 0, 0, 0, 0], [10, 2, 2, 1, 1])))
    assert e.value.status == mc.E_INVALID


def test_planned_tile_at_full_size_matches_plain_run():
    """The autotuner's tile for the full duct problem: same per-history
    results and tallies (to reordering) as the run without a tile."""
    mc = _mcdc()
    from paper_2409_04668_amd import autotune
    p = W.config2()
    tile, frac = autotune.plan_hot_tile(p, pilot=1_000_000)
    assert tile is not None and frac > 0.5
    n = 5_000_000
    res = []
    for opt in (mc.make_options(mc.SCHED_HISTORY), mc.make_options(mc.SCHED_HISTORY, tile=tile)):
        gp = mc.Problem(p, opt)
        gp.set_history_scores(n)
        gp.run(n, 77)
        res.append((gp.history_scores(), gp.raw()[0], gp.counters()))
        gp.close()
    assert np.array_equal(res[0][0], res[1][0])
    assert_close_sums(res[0][1], res[1][1], what="tally")
    assert res[0][2]["pieces"] == res[1][2]["pieces"]


# ---------------------------------------------------------------------------
# collision-estimator mesh tally
# ---------------------------------------------------------------------------

def _col_box():
    p = W._base(1)
    p["outer_lo"] = np.zeros(3)
    p["outer_hi"] = np.full(3, 10.0)
    p["box_lo"] = np.array([[4.0, 0.0, 0.0]])
    p["box_hi"] = np.array([[7.0, 10.0, 10.0]])
    p["box_mat"] = np.array([1], np.int32)
    p["sigma_t"] = np.array([[0.4], [1.5]])
    p["sigma_s"] = np.array([[[0.3]], [[1.2]]])
    p["source"] = dict(kind="box", lo=np.array([1.0, 1.0, 1.0]), hi=np.array([9.0, 9.0, 9.0]),
                       t0=0.0, t1=3.0, isotropic=True, dir=np.array([1.0, 0.0, 0.0]), group=0)
    p["mesh"] = dict(lo=np.array([2.0, 0.0, 1.0, 0.0]), hi=np.array([9.0, 10.0, 8.0, 8.0]),
                     n=np.array([7, 4, 5, 6], np.int32), per_group=False)
    p["census"] = np.array([5.0, 12.0])
    p["n_batches"] = 3
    p["collision_tally"] = True
    return p


def test_collision_tally_parity_history():
    gp, orc = full_parity(_col_box(), 3000, seed=131, trace_cap=300000)
    assert orc.col_sum.sum() > 0


def test_collision_tally_parity_event_and_multigroup_implicit():
    p = W.config3()
    p["implicit_capture"] = True
    p["mesh"]["n"] = np.array([6, 10, 6, 5], np.int32)
    p["collision_tally"] = True
    full_parity(p, 300, seed=132, trace_cap=600000, options=_ev())
    full_parity(p, 300, seed=133, trace_cap=600000)


def test_collision_tally_parity_duct_census_event_chunks():
    p = W.config2(n_census=5)
    p["mesh"]["n"] = np.array([12, 20, 12, 10], np.int32)
    p["collision_tally"] = True
    full_parity(p, 4321, seed=134, trace_cap=300000, options=_ev(1000))


def test_collision_tally_agrees_with_track_length_on_gpu():
    """1e7 duct histories: the two estimators of the same flux agree per bin
    within their statistical errors."""
    mc = _mcdc()
    p = W.config2()
    p["mesh"]["n"] = np.array([12, 20, 12, 4], np.int32)
    p["collision_tally"] = True
    gp = mc.Problem(p)
    gp.run(10_000_000, 135)
    mt, rt = gp.tallies(mc.TALLY_MESH)
    mcol, rc = gp.tallies(mc.TALLY_COLLISION)
    ok = (mt > 0) & (mcol > 0) & np.isfinite(rt) & np.isfinite(rc)
    assert ok.sum() > 500
    z = np.abs(mt - mcol)[ok] / np.hypot(mt * rt, mcol * rc)[ok]
    assert np.mean(z < 3) > 0.95 and np.max(z) < 6
    gp.close()


# ---------------------------------------------------------------------------
# population control at census (event schedule)
# ---------------------------------------------------------------------------

def _pc_pair(p, n, seed, chunk=0, trace_cap=400000):
    """Event-schedule run against the oracle: identical trajectories; the
    per-history sums of a history whose particles were split are compared to
    1e-12 (several particles add into them in another order)."""
    from gpu_util import assert_counters, assert_traces_equal
    gp, orc, tg, to, hg, ho = run_pair(p, n, seed, trace_cap=trace_cap, options=_ev(chunk))
    assert_traces_equal(tg[0], to[0])
    np.testing.assert_allclose(hg[0], ho[0], rtol=1e-12, atol=1e-300)
    s, s2 = gp.raw()
    assert_close_sums(s, orc.tally_sum, what="tally_sum")
    assert_close_sums(s2, orc.tally_sumsq, what="tally_sumsq")
    assert_counters(gp.counters(), orc)
    return gp, orc


def _void_pulse(target):
    p = W._base(1)
    p["outer_lo"] = np.full(3, -50.0)
    p["outer_hi"] = np.full(3, 50.0)
    p["sigma_t"] = np.array([[0.0]])
    p["sigma_s"] = np.array([[[0.0]]])
    p["mesh"] = dict(lo=np.array([-50.0, -50.0, -50.0, 0.0]), hi=np.array([50.0, 50.0, 50.0, 10.0]),
                     n=np.array([2, 1, 1, 5], np.int32), per_group=False)
    p["census"] = np.array([5.0, 10.0])
    p["n_batches"] = 2
    p["population_control"] = dict(target=target)
    return p


@pytest.mark.parametrize("target", [2.0, 0.3])
def test_population_control_parity_void(target):
    gp, orc = _pc_pair(_void_pulse(target), 1000, 141)
    c = orc.counters
    assert c["pc_copy"] > 0 if target > 1 else c["pc_kill"] > 0


def test_population_control_parity_infinite_medium():
    p = W.infinite_medium(1.0, [[0.9]], [1.0], half=5.0, t_end=8.0, nt=8)
    p["census"] = np.linspace(1.0, 8.0, 8)
    p["population_control"] = dict(target=1.5)
    p["n_batches"] = 4
    gp, orc = _pc_pair(p, 2000, 142)
    # analog weights stay 1 and the census population falls below the target,
    # so the control only splits
    assert orc.counters["pc_copy"] > 100


def test_population_control_parity_duct_with_weight_window_map():
    p = W.config2(n_census=4)
    p["mesh"]["n"] = np.array([6, 10, 6, 4], np.int32)
    p["ww"] = dict(params=ramp_mlp(-1.5, noise_seed=5), hidden=64, logk=0.3, ratio=5.0, n_max=10,
                   map=(12, 20, 12, 10))
    p["stack_cap"] = 256
    p["population_control"] = dict(target=0.7)
    gp, orc = _pc_pair(p, 1500, 143)
    assert orc.counters["pc_kill"] > 0 and orc.counters["split"] > 0


def test_population_control_rejections():
    mc = _mcdc()
    p = _void_pulse(1.0)
    with pytest.raises(mc.McdcError):
        mc.Problem(p, mc.make_options(mc.SCHED_HISTORY))
    gp = mc.Problem(p, _ev(100))                # batches of 500 histories do not fit
    with pytest.raises(mc.McdcError):
        gp.run(1000, 1)
    gp.close()


def test_population_control_unbiased_at_scale():
    """2e6 histories, eight census steps, target 0.5 per history: mesh tally
    of the controlled run agrees with the uncontrolled one."""
    mc = _mcdc()
    p = W.infinite_medium(1.0, [[0.8]], [1.0], half=20.0, t_end=8.0, nt=8)
    p["census"] = np.linspace(1.0, 8.0, 8)
    q = dict(p, population_control=dict(target=0.5))
    n = 2_000_000
    out = []
    for prob, seed in ((p, 151), (q, 152)):
        gp = mc.Problem(prob, _ev(1 << 20))
        gp.run(n, seed)
        out.append(gp.tallies(mc.TALLY_MESH))
        c = gp.counters()
        gp.close()
    (ma, ra), (mp, rp) = out
    z = np.abs(ma - mp) / np.hypot(ma * ra, mp * rp)
    assert np.all(z < 4.5), z
    assert c["pc_kills"] > 0


# ---------------------------------------------------------------------------
# edge cases: ragged and empty runs in the event schedule, maximum sizes
# ---------------------------------------------------------------------------

def test_ragged_and_empty_runs_event_schedule():
    p = W.config1()
    # fewer histories than batches, chunks of 4 histories, continuing ids
    for n in (0, 1, 7):
        full_parity(p, n, seed=113, trace_cap=1000, options=_ev(4))
    full_parity(p, 333, seed=114, trace_cap=20000, options=_ev(100), runs=3)
    # population control with batches of 3 and 4 histories
    _pc_pair(_void_pulse(2.0), 7, 115, chunk=8)


def test_largest_hot_tile_and_most_groups():
    """The largest LDS tile (19456 bins) on the duct, and eight energy groups
    (the most the library takes) with a per-group mesh."""
    mc = _mcdc()
    p = W.config2(n_census=2)
    tile = ([0, 0, 0, 0, 0], [16, 19, 16, 4, 1])
    assert int(np.prod(tile[1])) == mc.MAX_TILE_BINS
    full_parity(p, 3000, seed=116, trace_cap=200000, options=mc.make_options(tile=tile))
    q = W.config3()
    G = 8
    rng = np.random.default_rng(5)
    st = rng.uniform(0.05, 0.5, size=(3, G))
    ss = np.zeros((3, G, G))
    for m in range(3):
        for g in range(G):
            wts = rng.uniform(0.0, 1.0, size=g + 1)
            ss[m, g, :g + 1] = 0.7 * st[m, g] * wts / wts.sum()
    q["sigma_t"], q["sigma_s"] = st, ss
    q["speed"] = 10.0 ** (1.0 + np.arange(G) / 2.0)
    q["source"]["group"] = G - 1
    q["mesh"]["n"] = np.array([6, 10, 6, 4], np.int32)
    full_parity(q, 300, seed=117, trace_cap=600000)
    r = dict(q)
    r["sigma_t"] = np.ones((3, G + 1))
    r["sigma_s"] = np.zeros((3, G + 1, G + 1))
    r["speed"] = np.ones(G + 1)
    with pytest.raises(mc.McdcError):
        mc.Problem(r)


# ---------------------------------------------------------------------------
# stepped runs with checkpoint/resume
# ---------------------------------------------------------------------------

def _stepped_with_checkpoint(p, n, seed, opt, stop_after=2):
    """Begin a run, take `stop_after` steps, copy the workspace, the run
    record and the per-history output array into a fresh handle, and step
    that one to the end."""
    mc = _mcdc()
    ga = mc.Problem(p, opt)
    ga.set_history_scores(n)
    ga.run_begin(n, seed)
    for _ in range(stop_after):
        assert not ga.run_step()
    st = ga.run_state()
    assert st.in_run == 1 and st.steps == stop_after
    ws = ga.ws.clone()
    xh = ga._xh.clone()
    ga.close()
    gb = mc.Problem(p, opt)
    assert gb.ws.numel() == ws.numel()
    gb.ws.copy_(ws)
    gb.set_run_state(st)
    gb.set_history_scores(n)
    gb._xh.copy_(xh)
    steps = stop_after
    while not gb.run_step():
        steps += 1
        assert steps < 200
    return gb, steps + 1, st


def _check_stepped_against_oracle(gb, p, n, seed, exact_scores=True):
    orc = O.OracleRun(p)
    _, ho = orc.run(n, seed, per_history=True)
    if exact_scores:
        assert np.array_equal(gb.history_scores(), ho)
    else:
        np.testing.assert_allclose(gb.history_scores(), ho, rtol=1e-12, atol=1e-300)
    s, s2 = gb.raw()
    assert_close_sums(s, orc.tally_sum, what="tally_sum")
    assert_close_sums(s2, orc.tally_sumsq, what="tally_sumsq")
    if p.get("collision_tally"):
        c, _ = gb.raw_collision()
        assert_close_sums(c, orc.col_sum, what="col_sum")
    from gpu_util import assert_counters
    assert_counters(gb.counters(), orc)
    return orc


def test_census_steps_checkpoint_resume_matches_oracle():
    p = W.config2(n_census=5)
    p["mesh"]["n"] = np.array([12, 20, 12, 10], np.int32)
    p["collision_tally"] = True
    n, seed = 4000, 161
    gb, steps, _ = _stepped_with_checkpoint(p, n, seed, _ev(1 << 13))
    assert 3 <= steps <= 6
    _check_stepped_against_oracle(gb, p, n, seed)
    gb.close()


@pytest.mark.parametrize("hybrid", [False, True])
def test_stepped_run_over_several_resident_chunks(hybrid):
    """4500 histories with 1000 resident: five chunks (the last one ragged),
    each taken census step by census step, under three batches whose edges
    fall inside chunks; checkpointed inside the second or third chunk and
    resumed in a fresh handle."""
    mc = _mcdc()
    p = W.config2(n_census=3)
    p["mesh"]["n"] = np.array([12, 20, 12, 10], np.int32)
    p["n_batches"] = 3
    p["collision_tally"] = True
    n, seed = 4500, 163
    opt = mc.make_options(mc.SCHED_HYBRID if hybrid else mc.SCHED_EVENT, event_chunk=1000)
    ga = mc.Problem(p, opt)
    ga.run_begin(n, seed)
    per_chunk = 0
    while ga.run_state().segment == 0:
        assert not ga.run_step()
        per_chunk += 1
    ga.close()
    # a chunk takes one step per census step that some particle of it reaches
    assert 2 <= per_chunk <= 4
    gb, steps, st = _stepped_with_checkpoint(p, n, seed, opt, stop_after=2 * per_chunk + 1)
    assert 1 <= st.segment <= 2
    assert 5 * 2 <= steps <= 5 * 4
    _check_stepped_against_oracle(gb, p, n, seed)
    c = gb.counters()
    assert c["batches"] == 3 and c["histories"] == n
    gb.close()


def test_census_steps_checkpoint_resume_with_population_control():
    p = W.infinite_medium(1.0, [[0.9]], [1.0], half=5.0, t_end=8.0, nt=8)
    p["census"] = np.linspace(1.0, 8.0, 8)
    p["population_control"] = dict(target=1.5)
    p["n_batches"] = 1
    n, seed = 3000, 162
    gb, steps, _ = _stepped_with_checkpoint(p, n, seed, _ev(1 << 12), stop_after=3)
    assert steps == 8
    _check_stepped_against_oracle(gb, p, n, seed, exact_scores=False)
    gb.close()


@pytest.mark.parametrize("hybrid", [False, True])
def test_stepped_run_with_population_control_per_batch(hybrid):
    """Population control over three batches (1000, 1000, 1001 histories),
    each one resident chunk controlled on its own, as a plain run takes
    them; checkpointed inside the second batch (event schedule, or the
    hybrid schedule's lead and re-lead stages)."""
    mc = _mcdc()
    p = W.infinite_medium(1.0, [[0.9]], [1.0], half=5.0, t_end=8.0, nt=8)
    p["census"] = np.linspace(1.0, 8.0, 8)
    p["population_control"] = dict(target=1.5)
    p["n_batches"] = 3
    n, seed = 3001, 164
    opt = mc.make_options(mc.SCHED_HYBRID, event_chunk=1 << 11) if hybrid else _ev(1 << 11)
    gb, steps, st = _stepped_with_checkpoint(p, n, seed, opt, stop_after=10)
    assert st.segment == 1
    assert steps == 24
    orc = _check_stepped_against_oracle(gb, p, n, seed, exact_scores=False)
    assert orc.counters["pc_copy"] > 100
    gb.close()


def test_history_schedule_stepped_run_batch_by_batch():
    """Under the history schedule a step is one batch; checkpointed after two
    of four batches."""
    mc = _mcdc()
    p = W.config2(n_census=3)
    p["mesh"]["n"] = np.array([12, 20, 12, 10], np.int32)
    p["n_batches"] = 4
    p["collision_tally"] = True
    n, seed = 4001, 165
    gb, steps, st = _stepped_with_checkpoint(p, n, seed, mc.make_options(mc.SCHED_HISTORY))
    assert st.segment == 2 and steps == 4
    _check_stepped_against_oracle(gb, p, n, seed)
    assert gb.counters()["batches"] == 4
    gb.close()


def test_stepped_run_rejections():
    mc = _mcdc()
    p = W.config2(n_census=3)
    ge = mc.Problem(p, _ev(1000))
    with pytest.raises(mc.McdcError) as e:
        ge.run_step()                                # no run in progress
    assert e.value.status == mc.E_STATE
    with pytest.raises(mc.McdcError) as e:
        ge.run_begin(0, 1)                           # empty run
    assert e.value.status == mc.E_INVALID
    ge.run_begin(2500, 1)                            # three resident chunks
    with pytest.raises(mc.McdcError) as e:
        ge.run(10, 2)                                # a stepped run is in progress
    assert e.value.status == mc.E_STATE
    with pytest.raises(mc.McdcError) as e:
        ge.run_begin(10, 2)
    assert e.value.status == mc.E_STATE
    while not ge.run_step():
        pass
    ge.run(10, 2)                                    # and afterwards plain runs work again
    assert ge.counters()["histories"] == 2510
    st = ge.run_state()
    assert st.in_run == 0
    st.in_run = 1
    st.segment = 3                                   # the run had segments 0..2
    with pytest.raises(mc.McdcError) as e:
        ge.set_run_state(st)
    assert e.value.status == mc.E_INVALID
    with pytest.raises(mc.McdcError) as e:
        ge.run_step()                                # the bad record left no run in progress
    assert e.value.status == mc.E_STATE
    assert ge.counters()["histories"] == 2510       # and the handle as it was
    ge.close()
    q = W.infinite_medium(1.0, [[0.9]], [1.0], half=5.0, t_end=8.0, nt=8)
    q["population_control"] = dict(target=1.0)
    q["n_batches"] = 2
    gq = mc.Problem(q, _ev(1000))
    with pytest.raises(mc.McdcError) as e:
        gq.run_begin(2500, 1)                        # 1250 histories per controlled batch
    assert e.value.status == mc.E_INVALID
    gq.run_begin(2000, 1)
    while not gq.run_step():
        pass
    gq.close()


# ---------------------------------------------------------------------------
# weight windows with several energy groups (network input 4 + G)
# ---------------------------------------------------------------------------

def _ramp_mlp_g(in_dim, slope, group_bias, noise_seed=None):
    """y = slope * xhat_x + group_bias[g] (exact in FP32 up to the noise)."""
    H = 64
    prm = np.zeros(M.n_params(in_dim, H), np.float32)
    W1 = prm[:H * in_dim].reshape(H, in_dim)
    W1[0, 0] = 1.0                          # unit 0 carries xhat_x + 1
    for g, b in enumerate(group_bias):      # unit 1 + g carries the one-hot input of g
        W1[1 + g, 4 + g] = 1.0
    o = H * in_dim
    prm[o + 0] = 1.0                        # b1[0]
    o += H
    W2 = prm[o:o + H * H].reshape(H, H)
    W2[0, 0] = 1.0
    for g in range(len(group_bias)):
        W2[1 + g, 1 + g] = 1.0
    o += H * H + H
    prm[o + 0] = slope                      # W3
    for g, b in enumerate(group_bias):
        prm[o + 1 + g] = b
    o += H
    prm[o] = -slope                         # b3
    if noise_seed is not None:
        noise = M.init_params(in_dim, H, seed=noise_seed) * np.float32(0.01)
        prm = prm + noise
    return prm


@pytest.mark.parametrize("use_map", [False, True])
def test_weight_window_parity_multigroup(use_map):
    p = W.config3(n_census=2)
    p["mesh"]["n"] = np.array([6, 10, 6, 4], np.int32)
    G = 7
    ww = dict(params=_ramp_mlp_g(4 + G, -1.5, np.linspace(-1.0, 1.0, G), noise_seed=9), hidden=64,
              logk=0.5, ratio=5.0, n_max=10)
    if use_map:
        ww["map"] = (12, 20, 12, 8)
    p["ww"] = ww
    p["stack_cap"] = 256
    gp, orc = full_parity(p, 300, seed=171, trace_cap=800000)
    assert orc.counters["split"] > 10 and orc.counters["rr_kill"] > 10
    # the same histories under the event schedule
    from gpu_util import assert_counters, assert_traces_equal, run_pair
    ge, orc2, tg, to, hg, ho = run_pair(p, 300, 171, trace_cap=800000, options=_ev())
    assert_traces_equal(tg[0], to[0])
    np.testing.assert_allclose(hg[0], ho[0], rtol=1e-12, atol=1e-300)
    assert_counters(ge.counters(), orc2)


@pytest.mark.slow
def test_learned_ww_multigroup_pipeline_stays_unbiased():
    """Several groups: forward importance estimate, GPU training on 4 + G
    inputs, baked map, event schedule; the detector mean agrees with the
    analog run."""
    import math
    from paper_2409_04668_amd import learned_ww as L
    mc = _mcdc()
    # the duct problem in three groups (the 7-group data draw every region,
    # the duct too, from the same ranges, and then nothing reaches the
    # detector): shield and source Sigma_t near 0.1, a near-void duct,
    # downscatter with c = 0.5, speeds 1, 2, 4 cm/s
    p = W.config2()
    G = 3
    st = np.array([[0.10, 0.09, 0.11], [1e-4, 1e-4, 1e-4], [0.10, 0.08, 0.12]])
    ss = np.zeros((3, G, G))
    for m in range(3):
        for g in range(G):
            ss[m, g, :g + 1] = 0.5 * st[m, g] / (g + 1)
    p["sigma_t"], p["sigma_s"] = st, ss
    p["speed"] = np.array([1.0, 2.0, 4.0])
    p["source"]["group"] = G - 1
    p["mesh"] = dict(lo=np.array([0.0, 0.0, 0.0, 0.0]), hi=np.array([60.0, 100.0, 60.0, 200.0]),
                     n=np.array([6, 10, 6, 4], np.int32), per_group=True)
    ww, info = L.build_ww(p, n_runs=10, n_per_run=4_000_000, steps=800, map_dims=(12, 20, 12, 10))
    assert info["method"] == "forward" and info["loss_last"] < info["loss_first"]
    q = dict(p, ww=ww, stack_cap=256)
    out = []
    for prob, n, seed in ((p, 40_000_000, 181), (q, 8_000_000, 182)):
        gp = mc.Problem(prob, _ev(1 << 22))
        gp.run(n, seed)
        m, r = gp.tallies(mc.TALLY_DETECTOR)
        out.append((float(m[0]), float(r[0]) * float(m[0]), gp.counters()))
        gp.close()
    (ma, sa, _), (mw, sw, cw) = out
    assert ma > 0 and mw > 0
    assert abs(ma - mw) < 4 * math.hypot(sa, sw), out
    assert cw["splits"] > 0
