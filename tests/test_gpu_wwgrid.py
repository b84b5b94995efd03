"""GPU parity of the weight-window grid planes (a flight also stops on the
next interior plane of a grid over the outer box and the windows are checked
there) against the oracle, under the history, event and hybrid schedules:
identical traces (the plane stops among them), per-history sums to 1e-12
(split particles add in another order), tallies to 1e-10, counters exact."""
import numpy as np
import pytest

from paper_2409_04668_amd import workloads as W

from gpu_util import assert_close_sums, assert_counters, assert_traces_equal, run_pair
from test_gpu_parity import ramp_mlp
from test_oracle_wwgrid import _void_box

pytestmark = pytest.mark.gpu

SCHEDS = ["history", "event", "hybrid"]


def _opt(sched, chunk=0):
    from paper_2409_04668_amd import mcdc as mc
    return mc.make_options({"history": mc.SCHED_HISTORY, "event": mc.SCHED_EVENT,
                            "hybrid": mc.SCHED_HYBRID}[sched], event_chunk=chunk)


def _pair(p, n, seed, options, trace_cap=600000):
    gp, orc, tg, to, hg, ho = run_pair(p, n, seed, trace_cap=trace_cap, options=options)
    assert_traces_equal(tg[0], to[0])
    np.testing.assert_allclose(hg[0], ho[0], rtol=1e-12, atol=1e-300)
    s, s2 = gp.raw()
    assert_close_sums(s, orc.tally_sum, what="tally_sum")
    assert_close_sums(s2, orc.tally_sumsq, what="tally_sumsq")
    assert_counters(gp.counters(), orc)
    return gp, orc


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("direction", [(1.0, 0.0, 0.0), (-1.0, 0.0, 0.0)])
def test_void_beam_plane_stops(sched, direction):
    gp, orc = _pair(_void_box(direction), 300, 201, _opt(sched))
    assert orc.counters["ww_plane"] == 300 and orc.counters["split"] == 900


@pytest.mark.parametrize("sched", SCHEDS)
def test_plane_on_a_surface_yields(sched):
    gp, orc = _pair(_void_box((1.0, 0.0, 0.0), boxes=True), 300, 202, _opt(sched))
    assert orc.counters["ww_plane"] == 0 and orc.counters["split"] == 900


def _ramp_box(grid, use_map=False):
    p = W._base(1)
    p["outer_lo"] = np.zeros(3)
    p["outer_hi"] = np.full(3, 20.0)
    p["sigma_t"] = np.array([[0.3]])
    p["sigma_s"] = np.array([[[0.2]]])
    p["source"] = dict(kind="point", lo=np.full(3, 10.0), hi=np.full(3, 10.0), t0=0.0, t1=0.0,
                       isotropic=True, dir=np.array([1.0, 0.0, 0.0]), group=0)
    p["mesh"] = dict(lo=np.zeros(4), hi=np.array([20.0, 20.0, 20.0, 40.0]),
                     n=np.array([10, 4, 4, 4], np.int32), per_group=False)
    p["census"] = np.array([20.0, 40.0])
    p["ww"] = dict(params=ramp_mlp(2.0, noise_seed=3), hidden=64, logk=0.0, ratio=5.0, n_max=10,
                   ymin=-1.5, ymax=1.5, grid=grid, map=(10, 4, 4, 8) if use_map else None)
    return p


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("use_map", [False, True])
def test_ramp_windows_with_grid_planes(sched, use_map):
    gp, orc = _pair(_ramp_box((10, 4, 4), use_map), 1500, 203, _opt(sched))
    c = orc.counters
    assert c["ww_plane"] > 1000 and c["split"] > 100 and c["rr_kill"] > 20


def test_duct_with_map_grid_and_population_control_hybrid():
    p = W.config2(n_census=4)
    p["mesh"]["n"] = np.array([6, 10, 6, 4], np.int32)
    p["ww"] = dict(params=ramp_mlp(-1.5, noise_seed=5), hidden=64, logk=0.3, ratio=5.0, n_max=10,
                   map=(12, 20, 12, 10), grid=(12, 20, 12))
    p["population_control"] = dict(target=0.7)
    gp, orc = _pair(p, 1500, 204, _opt("hybrid"))
    assert orc.counters["ww_plane"] > 100 and orc.counters["pc_kill"] > 0


def test_grid_requires_a_network():
    from paper_2409_04668_amd import mcdc as mc
    p = W.config1()
    gp = mc.Problem(p)
    with pytest.raises(mc.McdcError):
        gp.set_ww_grid((4, 4, 4))
    gp.set_ww_grid(None)
    gp.close()
