"""GPU parity of the surface-current tally (weight of every flight crossing an
axis-aligned plane, by side, group, time and in-plane mesh bins) against the
oracle: per-history results bit-identical (one particle per history) or to
1e-12 (split particles), surface sums to 1e-10, the crossing count exact;
under the history, event and hybrid schedules, with census steps, per-group
meshes, a partial mesh, weight windows, population control and census-step
checkpoint/resume."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_04668_amd import workloads as W

from gpu_util import assert_close_sums, assert_counters, assert_traces_equal, full_parity, run_pair
from test_gpu_parity import _stepped_with_checkpoint, _void_pulse, ramp_mlp
from test_oracle_surface import _two_group_box

pytestmark = pytest.mark.gpu


def _mc():
    from paper_2409_04668_amd import mcdc
    return mcdc


def _opt(sched, chunk=0, tile=None):
    mc = _mc()
    return mc.make_options({"history": mc.SCHED_HISTORY, "event": mc.SCHED_EVENT,
                            "hybrid": mc.SCHED_HYBRID}[sched], event_chunk=chunk, tile=tile)


def _split_pair(p, n, seed, options, trace_cap=400000):
    gp, orc, tg, to, hg, ho = run_pair(p, n, seed, trace_cap=trace_cap, options=options)
    assert_traces_equal(tg[0], to[0])
    np.testing.assert_allclose(hg[0], ho[0], rtol=1e-12, atol=1e-300)
    s, s2 = gp.raw()
    assert_close_sums(s, orc.tally_sum, what="tally_sum")
    c, c2 = gp.raw_surface()
    assert_close_sums(c, orc.surf_sum, what="surf_sum")
    assert_close_sums(c2, orc.surf_sumsq, what="surf_sumsq")
    assert_counters(gp.counters(), orc)
    return gp, orc


@pytest.mark.parametrize("sched", ["history", "hybrid"])
def test_surface_tally_slab(sched):
    """The slab's y and z axes are unbounded: one in-plane bin."""
    p = W.config1()
    p["surface_tally"] = dict(axis=0, pos=0.5)
    gp, orc = full_parity(p, 3000, seed=191, trace_cap=60000, options=_opt(sched))
    assert orc.counters["surf_cross"] > 500


def test_surface_tally_duct_census_event_chunks():
    p = W.config2(n_census=5)
    p["mesh"]["n"] = np.array([12, 20, 12, 10], np.int32)
    p["surface_tally"] = dict(axis=1, pos=20.0)
    gp, orc = full_parity(p, 4321, seed=192, trace_cap=300000, options=_opt("event", 1000))
    assert orc.counters["surf_cross"] > 100


def test_surface_tally_multigroup_implicit_hybrid():
    p = W.config3()
    p["implicit_capture"] = True
    p["mesh"]["n"] = np.array([6, 10, 6, 5], np.int32)
    p["surface_tally"] = dict(axis=2, pos=5.0)
    gp, orc = full_parity(p, 300, seed=193, trace_cap=600000, options=_opt("hybrid"))
    assert orc.counters["surf_cross"] > 100


@pytest.mark.parametrize("sched", ["history", "event", "hybrid"])
def test_surface_tally_two_groups_partial_mesh(sched):
    p = _two_group_box()
    tile = ([1, 0, 0, 0, 0], [4, 4, 5, 3, 2]) if sched != "event" else None
    gp, orc = full_parity(p, 3000, seed=194, trace_cap=800000, options=_opt(sched, tile=tile))
    s = orc.surf_sum.reshape(2, 2, -1).sum(axis=2)
    assert np.all(s > 0)


def test_surface_tally_with_weight_window_map_hybrid():
    p = W.config2(n_census=3)
    p["mesh"]["n"] = np.array([6, 10, 6, 4], np.int32)
    p["ww"] = dict(params=ramp_mlp(-1.5, noise_seed=5), hidden=64, logk=0.3, ratio=5.0, n_max=10,
                   map=(12, 20, 12, 10))
    p["surface_tally"] = dict(axis=0, pos=8.0)
    gp, orc = _split_pair(p, 900, 195, _opt("hybrid", 256))
    assert orc.counters["split"] > 10 and orc.counters["surf_cross"] > 100


def test_surface_tally_with_population_control():
    p = _void_pulse(0.3)
    p["surface_tally"] = dict(axis=0, pos=3.0)
    gp, orc = _split_pair(p, 1000, 196, _opt("event"))
    assert orc.counters["pc_kill"] > 0 and orc.counters["surf_cross"] > 100


def test_surface_tally_census_steps_checkpoint_resume():
    p = W.config2(n_census=5)
    p["mesh"]["n"] = np.array([12, 20, 12, 10], np.int32)
    p["surface_tally"] = dict(axis=1, pos=20.0)
    n, seed = 4000, 197
    gb, steps, _ = _stepped_with_checkpoint(p, n, seed, _opt("hybrid", 1 << 13))
    orc = O.OracleRun(p)
    _, ho = orc.run(n, seed, per_history=True)
    assert np.array_equal(gb.history_scores(), ho)
    c, c2 = gb.raw_surface()
    assert_close_sums(c, orc.surf_sum, what="surf_sum")
    assert_close_sums(c2, orc.surf_sumsq, what="surf_sumsq")
    assert_counters(gb.counters(), orc)
    gb.close()


def test_surface_tally_means_are_per_area_and_time():
    """mcdc_get_tallies(MCDC_TALLY_SURFACE): the mean crossing weight per
    history divided by the bin's in-plane area and time width, with batch
    relative errors; the raw sums are the oracle's."""
    mc = _mc()
    p = W.config2()
    p["mesh"]["n"] = np.array([12, 20, 12, 10], np.int32)
    p["surface_tally"] = dict(axis=1, pos=45.0)
    n = 200_000
    gp = mc.Problem(p)
    gp.run(n, 198)
    mean, rel = gp.tallies(mc.TALLY_SURFACE)
    s, s2 = gp.raw_surface()
    lo, hi, nn = p["mesh"]["lo"], p["mesh"]["hi"], p["mesh"]["n"]
    dx = (hi[0] - lo[0]) / nn[0]
    dz = (hi[2] - lo[2]) / nn[2]
    dt = (hi[3] - lo[3]) / nn[3]
    np.testing.assert_allclose(mean, s / n / (dx * dz * dt), rtol=1e-14)
    hit = s > 0
    assert hit.sum() > 50 and np.all(np.isfinite(rel[hit])) and np.all(rel[hit] > 0)
    assert gp.surface_bins() == 2 * 10 * 12 * 12
    with pytest.raises(mc.McdcError):
        gp.raw_collision()
    gp.close()
    q = W.config2()
    gq = mc.Problem(q)
    gq.run(1000, 1)
    with pytest.raises(mc.McdcError):
        gq.raw_surface()
    gq.close()
